/*
 * CPU oracle core (TEST INFRASTRUCTURE ONLY: used by tests/, smoke() and the
 * bench's cpu_baseline leg; never by the GPU library).
 *
 * Plain, slow, obviously correct matrix elements of the shell-model
 * Hamiltonian (Sec. 2):
 *     H = sum_s e_s n_s + sum_{a<b, c<d} h_abcd c+_a c+_b c_d c_c
 * between Slater determinants held as one 64-bit word each (protons in the low
 * bits, neutrons above them). A determinant is c+_{s1} c+_{s2} ... |0> with
 * s1 < s2 < ..., so an operator on state s picks up (-1)^(number of occupied
 * states below s) (Jordan-Wigner order over the combined state index).
 *
 * Matrix element <i|c+_a c+_b c_d c_c|j> is found from the adjoint term
 * c+_c c+_d c_b c_a applied to |i> (App. B: bit operations, then a binary
 * search for the serial number of the resulting determinant).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static int jw_sign(uint64_t w, int s) {
    uint64_t below = (s == 0) ? 0 : (w & ((((uint64_t)1) << s) - 1));
    return (__builtin_popcountll(below) & 1) ? -1 : 1;
}

/* annihilate state s: returns 0 if empty */
static int ann(uint64_t* w, int s, int* sign) {
    uint64_t bit = ((uint64_t)1) << s;
    if (!(*w & bit)) return 0;
    *sign *= jw_sign(*w, s);
    *w &= ~bit;
    return 1;
}

/* create state s: returns 0 if occupied */
static int cre(uint64_t* w, int s, int* sign) {
    uint64_t bit = ((uint64_t)1) << s;
    if (*w & bit) return 0;
    *sign *= jw_sign(*w, s);
    *w |= bit;
    return 1;
}

static int64_t find(const uint64_t* sorted, const int64_t* idx, int64_t n, uint64_t w) {
    int64_t lo = 0, hi = n - 1;
    while (lo <= hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (sorted[mid] == w) return idx[mid];
        if (sorted[mid] < w) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

typedef struct { int64_t col; double val; } entry;

static int cmp_entry(const void* x, const void* y) {
    int64_t a = ((const entry*)x)->col, b = ((const entry*)y)->col;
    return (a > b) - (a < b);
}

/*
 * Non-zeros of row i (mode 0: <i|H|j> via adjoint terms, grouped by the
 * creation pair (a,b) = grp1,grp2) or of column i (mode 1: <j|H|i> via the
 * terms themselves, grouped by the annihilation pair (c,d)).
 * Terms k in [start[p*S+q], start[p*S+q+1]) have group pair (p,q).
 * Returns the number of merged entries written (<= cap), or -1 if cap is too small.
 * With merge == 0 the entries are left as generated: one per term that reaches a basis state,
 * plus the single-particle-energy diagonal first (a per-element sum adds exactly these).
 */
static int64_t line_entries(int mode, int64_t i, const uint64_t* words, const uint64_t* sorted,
                            const int64_t* sidx, int64_t D, int S, const double* e,
                            const int* ta, const int* tb, const int* tc, const int* td,
                            const double* th, const int64_t* start, entry* buf, int64_t cap, int merge) {
    uint64_t w = words[i];
    int64_t n = 0;
    double diag = 0.0;
    for (int s = 0; s < S; s++)
        if (w & (((uint64_t)1) << s)) diag += e[s];
    buf[n].col = i; buf[n].val = diag; n++;
    for (int p = 0; p < S; p++) {
        if (!(w & (((uint64_t)1) << p))) continue;
        for (int q = p + 1; q < S; q++) {
            if (!(w & (((uint64_t)1) << q))) continue;
            for (int64_t k = start[p * S + q]; k < start[p * S + q + 1]; k++) {
                uint64_t x = w;
                int sign = 1;
                int a = ta[k], b = tb[k], c = tc[k], d = td[k];
                int ok;
                if (mode == 0) /* c+_c c+_d c_b c_a |i> */
                    ok = ann(&x, a, &sign) && ann(&x, b, &sign) && cre(&x, d, &sign) && cre(&x, c, &sign);
                else           /* c+_a c+_b c_d c_c |i> */
                    ok = ann(&x, c, &sign) && ann(&x, d, &sign) && cre(&x, b, &sign) && cre(&x, a, &sign);
                if (!ok) continue;
                int64_t j = find(sorted, sidx, D, x);
                if (j < 0) continue; /* outside the M (and parity) block: cannot happen for scalar H */
                if (n >= cap) return -1;
                buf[n].col = j; buf[n].val = th[k] * sign; n++;
            }
        }
    }
    if (!merge) return n;
    qsort(buf, (size_t)n, sizeof(entry), cmp_entry);
    int64_t m = 0;
    for (int64_t t = 0; t < n; t++) {
        if (m > 0 && buf[m - 1].col == buf[t].col) buf[m - 1].val += buf[t].val;
        else buf[m++] = buf[t];
    }
    return m;
}

/* Rows (mode 0) or columns (mode 1) of H for the listed indices, as CSR pieces (merge == 0:
   the generated terms, unmerged). out_ptr has nlist+1 entries; returns 0, or -1 if cap_total is
   exceeded. */
int orc_lines(int mode, const int64_t* list, int64_t nlist, const uint64_t* words,
              const uint64_t* sorted, const int64_t* sidx, int64_t D, int S, const double* e,
              const int* ta, const int* tb, const int* tc, const int* td, const double* th,
              const int64_t* start, int64_t per_line_cap, int64_t* out_ptr, int64_t* out_col,
              double* out_val, int64_t cap_total, int merge) {
    entry* buf = (entry*)malloc(sizeof(entry) * (size_t)per_line_cap);
    if (!buf) return -2;
    out_ptr[0] = 0;
    for (int64_t r = 0; r < nlist; r++) {
        int64_t m = line_entries(mode, list[r], words, sorted, sidx, D, S, e, ta, tb, tc, td, th,
                                 start, buf, per_line_cap, merge);
        if (m < 0 || out_ptr[r] + m > cap_total) { free(buf); return -1; }
        for (int64_t t = 0; t < m; t++) {
            out_col[out_ptr[r] + t] = buf[t].col;
            out_val[out_ptr[r] + t] = buf[t].val;
        }
        out_ptr[r + 1] = out_ptr[r] + m;
    }
    free(buf);
    return 0;
}

/* W[r, :] = sum_j H[list[r], j] V[j, :] for nb columns (row-major V: D x nb).
   Rows are independent; OpenMP splits them over threads. */
int orc_apply_rows(const int64_t* list, int64_t nlist, const uint64_t* words, const uint64_t* sorted,
                   const int64_t* sidx, int64_t D, int S, const double* e, const int* ta,
                   const int* tb, const int* tc, const int* td, const double* th,
                   const int64_t* start, int64_t per_line_cap, const double* V, int nb, double* W) {
    int err = 0;
#pragma omp parallel
    {
        entry* buf = (entry*)malloc(sizeof(entry) * (size_t)per_line_cap);
        if (!buf) {
#pragma omp atomic write
            err = -2;
        } else {
#pragma omp for schedule(dynamic, 64)
            for (int64_t r = 0; r < nlist; r++) {
                int64_t m = line_entries(0, list[r], words, sorted, sidx, D, S, e, ta, tb, tc, td,
                                         th, start, buf, per_line_cap, 1);
                double* out = W + r * (int64_t)nb;
                for (int c = 0; c < nb; c++) out[c] = 0.0;
                if (m < 0) {
#pragma omp atomic write
                    err = -1;
                    continue;
                }
                for (int64_t t = 0; t < m; t++) {
                    const double* vin = V + buf[t].col * (int64_t)nb;
                    double h = buf[t].val;
                    for (int c = 0; c < nb; c++) out[c] += h * vin[c];
                }
            }
            free(buf);
        }
    }
    return err;
}

/* Number of non-zero elements of every listed row (structural count after merging). */
int orc_row_nnz(const int64_t* list, int64_t nlist, const uint64_t* words, const uint64_t* sorted,
                const int64_t* sidx, int64_t D, int S, const double* e, const int* ta, const int* tb,
                const int* tc, const int* td, const double* th, const int64_t* start,
                int64_t per_line_cap, int64_t* nnz) {
    int err = 0;
#pragma omp parallel
    {
        entry* buf = (entry*)malloc(sizeof(entry) * (size_t)per_line_cap);
        if (!buf) {
#pragma omp atomic write
            err = -2;
        } else {
#pragma omp for schedule(dynamic, 256)
            for (int64_t r = 0; r < nlist; r++) {
                int64_t m = line_entries(0, list[r], words, sorted, sidx, D, S, e, ta, tb, tc, td, th,
                                         start, buf, per_line_cap, 1);
                nnz[r] = m;
                if (m < 0) {
#pragma omp atomic write
                    err = -1;
                }
            }
            free(buf);
        }
    }
    return err;
}

int orc_num_threads(void) {
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
