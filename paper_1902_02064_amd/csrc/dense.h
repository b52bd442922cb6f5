// Declarations of the dense block kernels (dense.hip) used by the TRBL driver.
#pragma once
#include <algorithm>

#include "internal.h"

namespace trbl {

// Grow-only device scratch for per-workgroup partial sums.
struct Scratch {
  DevBuf buf;
  int last_G = 0;
  double* last_part = nullptr;
  double* partials(size_t n) {
    buf.alloc(n * sizeof(double));
    return buf.as<double>();
  }
};

// C (m x nb) = A^T B over D rows.
template <class TA, class TB>
void tn(const TA* A, int64_t lda, int m, const TB* B, int64_t ldb, int nb, int64_t D, double* C, Scratch& s,
        hipStream_t st);
// Bout = Bin - A C; mode 1 also forms A^T Bout into Pout, mode 2 keeps Bout^T Bout partials in s
// (of the stored values; FP32 Bout: modes 0 and 2 only). Modes 0 and 2 may store the same
// values a second time into Bout2 (leading dimension ldo2).
template <class TA, class TI, class TO = double>
void update(const TA* A, int64_t lda, int m, const double* C, const TI* Bin, int64_t ldi, TO* Bout, int64_t ldo,
            int nb, int64_t D, int mode, double* Pout, Scratch& s, hipStream_t st, TO* Bout2 = nullptr,
            int64_t ldo2 = 0);
// Bout = Bin R (R nb x nb); gram keeps Bout^T Bout partials in s; optional second copy in Bout2.
template <class TI, class TO>
void apply_small(const TI* Bin, int64_t ldi, const double* R, TO* Bout, int64_t ldo, int nb, int64_t D, bool gram,
                 Scratch& s, hipStream_t st, TO* Bout2 = nullptr, int64_t ldo2 = 0);
// Cholesky of the sum of G partial nb x nb Gram matrices: R, R^-1, beta = R Rprev (if beta), status.
void chol(const double* part, int G, int nb, double* R, double* Rinv, const double* Rprev, double* beta, int* status,
          hipStream_t st);
// Y[:, 0:ncol] = A[:, 0:m] U (row-wise, in place allowed); then optional column block move
// (columns [vsrc, vsrc+nv) of A to [vdst, vdst+nv) of Y). In place with ncol > 208 needs a work
// buffer tmp of tmp_elems >= ncol + nv elements (rows go through it in chunks; vdst >= ncol).
template <class TA, class TY>
void rowgemm(const TA* A, int64_t lda, int m, const double* U, int64_t ldu, int ncol, TY* Y, int64_t ldy, int64_t D,
             int vsrc, int vdst, int nv, hipStream_t st, TY* tmp = nullptr, int64_t tmp_elems = 0);
template <class T>
void random_block(T* out, int64_t ld, int64_t D, int nb, uint64_t seed, hipStream_t st);
template <class TS, class TD>
void copy_cols(const TS* src, int64_t lds_, TD* dst, int64_t ldd, int64_t D, int ncol, hipStream_t st);
// X[r, 0:ncol] = 0 where mask[r] == 0 (no-op for a null mask)
template <class T>
void mask_rows(T* X, int64_t ld, int64_t D, int ncol, const double* mask, hipStream_t st);
void t_alpha(double* T, int ldt, int c0, int nb, const double* C1, hipStream_t st);
// C[r, :] = T[r, c0:c0+nb] for r in [r_lo, c0) (C row-major, nb columns)
void t_column(const double* T, int ldt, int c0, int r_lo, int nb, double* C, hipStream_t st);
void t_beta(double* T, int ldt, int c0, int m, int nb, const double* beta, hipStream_t st);
void resid(const double* beta, int nb, const double* U, int ldu, int m, int n, double* rho, hipStream_t st);
void t_restart(double* T, int ldt, int lm, const double* theta, int ls, const double* beta, int nb, const double* U,
               int ldu, int m, hipStream_t st);

constexpr int EIG_NMAX = 640;  // largest projected matrix the device eigensolver takes

// Symmetric eigensolver of a small dense matrix (eig.hip): all eigenvalues ascending in theta[0:n],
// orthonormal eigenvectors of the nvec lowest in U (n x nvec, ld ldu).
struct EigWork {
  DevBuf a, z, lu, aux, xb, flag;
};
void symeig(const double* T, int ldt, int n, int nvec, double* theta, double* U, int ldu, EigWork& w, bool orth,
            hipStream_t st);
// Generalised problem S y = theta G y (G positive definite, n x n): M = L^-1 S L^-T into M, L^-1 into Linv.
void gen_reduce(const double* S, const double* G, int n, double* M, double* Linv, int* status, hipStream_t st);
// Y = L^-T Yp (n x nv, ld ldy).
void gen_back(const double* Linv, const double* Yp, int ldp, int n, int nv, double* Y, int ldy, hipStream_t st);
// out[c] = sum_r W[r, c] X[r, c] over D rows (device out, ncol <= 64); part holds dot_cols_parts(D) * ncol
// doubles of partial sums
int dot_cols_parts(int64_t D);
void dot_cols(const double* W, int64_t ldw, const double* X, int64_t ldx, int ncol, int64_t D, double* part,
              double* out, hipStream_t st);
// column norms of W - X diag(theta) over D rows: out[c] (squared sums accumulated, then sqrt on host side)
void resid_cols(const double* W, int64_t ldw, const double* X, int64_t ldx, const double* theta, int ncol, int64_t D,
                double* out, Scratch& s, hipStream_t st);

}  // namespace trbl
