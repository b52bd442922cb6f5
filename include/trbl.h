/*
 * trbl.h -- C ABI of libtrbl: thick-restart block Lanczos (TRBL) for the
 * M-scheme nuclear shell model on one AMD Instinct MI355X (gfx950).
 *
 * Method: Shimizu, Mizusaki, Utsuno, Tsunoda, "Thick-restart block Lanczos
 * method for large-scale shell-model calculations" (arXiv:1902.02064).
 *   - model space and basis: Sec. 2 (M-scheme Slater determinants as bit
 *     strings) and App. A (Table 1 ordering, partitions, proton x neutron
 *     product form);
 *   - Hamiltonian: Sec. 2 (one-body + two-body operator with J-coupled
 *     two-body matrix elements);
 *   - H applied to a block of vectors on the fly: App. B (identical-particle
 *     two-body jumps; proton-neutron factorisation through one-body jumps);
 *   - eigensolver: Alg. 4 and the thick-restart equations of Sec. 3.4;
 *   - single-species spaces and start vectors from a particle-hole truncated
 *     space: Sec. 4.2 (trbl_occupation_mask, trbl_opts.mask).
 *
 * Conventions (fixed by this header):
 *   - Single-particle m-states of one species: orbits in the order given,
 *     then 2m ascending (Table 1 column order); bit s of a 64-bit word is
 *     state s. At most 64 m-states per species.
 *   - Species sectors (2M_s, parity): occupation partitions in descending
 *     lexicographic order; inside a partition, occupied-state tuples in
 *     ascending lexicographic order (this is exactly Table 1).
 *   - Product basis: blocks ordered by 2M_p ascending, then proton parity
 *     + before -, then neutron parity + before -; inside a block,
 *     index = block offset + p * D_n + n  (proton-major).
 *   - Vectors: row-major [D][nb] (element (i, c) at i*nb + c), FP64
 *     (TRBL_FP64) or FP32 (TRBL_MIXED), caller-owned device memory.
 *   - Two-body matrix elements: proton-neutron formalism, normalised and
 *     antisymmetrised J-coupled elements V_J(ab,cd) with Condon-Shortley
 *     Clebsch-Gordan coefficients, orbit a coupled before b (proton before
 *     neutron in the pn channel). Each independent element is listed once;
 *     the mirror V_J(cd,ab) is implied. An identical-particle pair given as
 *     (b,a) is reordered with V_J(ba,cd) = -(-1)^(ja+jb-J) V_J(ab,cd).
 *
 * Errors: every int-returning call returns 0 on success, a negative
 * TRBL_E* code on failure (message from trbl_last_error(), thread-local),
 * or TRBL_NOT_CONVERGED (+1) from trbl_solve, which still writes the best
 * Ritz pairs. No C++ exception crosses this boundary.
 * Threading: one model may be used by one host thread / stream at a time.
 */
#ifndef TRBL_H
#define TRBL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TRBL_OK 0
#define TRBL_NOT_CONVERGED 1
#define TRBL_E_INVALID (-1)   /* bad argument */
#define TRBL_E_EMPTY (-2)     /* empty model space (D = 0) */
#define TRBL_E_TOO_MANY (-3)  /* more than 64 m-states per species */
#define TRBL_E_NOMEM (-4)     /* host or device allocation failed */
#define TRBL_E_DEVICE (-5)    /* HIP runtime error */
#define TRBL_E_BREAKDOWN (-6) /* unrecoverable breakdown: no direction left outside the basis */
#define TRBL_E_STATE (-7)     /* call order (e.g. no Hamiltonian set) */

typedef struct trbl_model trbl_model; /* opaque, library-owned */

typedef enum { TRBL_FP64 = 0, TRBL_MIXED = 1 } trbl_precision;
typedef enum { TRBL_CONV_RESIDUAL = 0, TRBL_CONV_RITZ_CHANGE = 1 } trbl_criterion;

typedef struct {
  int n, l, twoj; /* radial number, orbital l, 2j */
} trbl_orbit;

typedef struct {
  int channel;    /* 0 = pp, 1 = nn, 2 = pn (a, c proton orbits; b, d neutron orbits) */
  int a, b, c, d; /* orbit indices into the model's orbit list */
  int twoJ;       /* 2J of the pair */
  double v;       /* V_J(ab,cd) */
} trbl_tbme;

typedef struct {
  int nb;          /* block size p (1..64) */
  int n_eig;       /* wanted lowest eigenpairs N */
  int l_s;         /* vectors kept at a thick restart (N <= l_s) */
  int l_m;         /* maximum stored Lanczos vectors (l_s + 2*nb <= l_m <= D, l_m - nb <= 640) */
  int max_iter;    /* block iterations before giving up */
  double tol;      /* residual tolerance: rho_i <= tol * max|theta| */
  int precision;   /* trbl_precision */
  int refine;      /* mixed mode: 1 = final FP64 Rayleigh-Ritz refinement */
  uint64_t seed;   /* seed of the random start block (splitmix64 + Box-Muller) */
  const void* v0;  /* optional device start block [D][nb] (FP64 or FP32 per precision); NULL = random */
  void* stream;    /* hipStream_t; NULL = default stream */
  int check_every; /* diagonalise T for the convergence test every k iterations (and at every
                      restart); 0 or 1 = every iteration, as in Alg. 4; negative = adaptive:
                      the next test is scheduled from the observed decay of the largest
                      residual (every restart still tests) */
  int criterion;   /* TRBL_CONV_RESIDUAL (0): rho_i <= tol * max|theta|;
                      TRBL_CONV_RITZ_CHANGE (1): the paper's test of Sec. 4.1, the n_eig lowest Ritz
                      values move by at most tol (absolute) between two consecutive tests */
  const double* mask; /* optional device [D] of 0/1 (e.g. from trbl_occupation_mask); NULL = none.
                      When set the solve works in the subspace of the basis states with mask 1:
                      H is replaced by P H P (P = diag(mask)), the start block and every
                      replacement vector are projected, so eigenpairs of the truncated space
                      come out (start vectors of Sec. 4.2). Must stay valid during the call. */
} trbl_opts;

typedef struct {
  int iterations, restarts, n_converged, breakdowns;
  double t_total, t_hv, t_orth, t_qr, t_eig, t_restart, t_refine; /* seconds (device events) */
  double* resid;   /* optional caller host buffer of n_eig residual norms ||H x - theta x|| of the
                      returned pairs, computed with H itself in FP64 */
} trbl_info;

/* Build the M-scheme product basis (Sec. 2, App. A). parity: +1, -1, or 0 for both.
   Copies the orbit list. *out owns host and device tables until trbl_model_destroy.
   With one species empty (single-species spaces of Sec. 4.2) only the sectors of the other
   species that form the space are enumerated; when the widest of them exceeds 2048
   determinants (or the environment variable TRBL_FLY is "1" at this call) the products
   generate the identical-particle part per element instead of storing it, which needs at most
   44 m-states and keeps two [D][nb] work blocks per precision with the model. */
int trbl_model_create(const trbl_orbit* orbits, int n_orbits, int n_prot, int n_neut, int twoM,
                      int parity, trbl_model** out);
void trbl_model_destroy(trbl_model* m);

/* M-scheme dimension D. */
int trbl_model_dim(const trbl_model* m, int64_t* dim);

/* Host-side index <-> bit strings (App. A, Table 1 order). rank writes -1 for a state outside the basis. */
int trbl_basis_unrank(const trbl_model* m, int64_t i, uint64_t* pbits, uint64_t* nbits);
int trbl_basis_rank(const trbl_model* m, uint64_t pbits, uint64_t nbits, int64_t* i);

/* Device-side bulk versions (GPU kernels): idx, pbits, nbits are device arrays of length n. */
int trbl_basis_unrank_dev(const trbl_model* m, const int64_t* idx, int64_t n, uint64_t* pbits,
                          uint64_t* nbits, void* stream);
int trbl_basis_rank_dev(const trbl_model* m, const uint64_t* pbits, const uint64_t* nbits, int64_t n,
                        int64_t* idx, void* stream);

/* The seeded synthetic interaction of the benchmark workloads (a stand-in for the tabulated
   interactions the paper uses with the Hamiltonian of Sec. 2): every independent J-coupled
   element V_J(ab,cd) of the pp, nn and pn channels drawn i.i.d. from N(0, sigma^2), as
   trbl_set_hamiltonian takes them. Order: channel pp, nn, pn; 2J = 0, 2, ..., 2 * (largest 2j);
   pair parity + then -; inside a (channel, 2J, parity) block the allowed pairs (a <= b for pp
   and nn, every (a, b) for pn; orbit order) and all pairs (i <= j) of them. Draw k is
   sigma * sqrt(-2 ln u1) cos(2 pi u2), u1 = u(2k), u2 = u(2k + 1), u(c) = ((s >> 11) + 1) / 2^53
   with s the c-th output of splitmix64 from state seed. Host only (no device needed).
   out: host array of `capacity` elements, or NULL (with capacity 0) to ask for the count;
   *n_out = the number of elements. TRBL_E_INVALID for a bad orbit or a short buffer. */
int trbl_random_tbme(const trbl_orbit* orbits, int n_orbits, uint64_t seed, double sigma, trbl_tbme* out,
                     int64_t capacity, int64_t* n_out);

/* Set H = sum_a e_a n_a + two-body (Sec. 2). spe_p, spe_n: one energy per orbit (host).
   tbme: n_v host elements. Copies everything, builds the one-body jump and
   identical-particle tables of App. B on the device. Where it fits in a quarter of the free
   device memory (and below 4 GiB for two species), and for two species where a core pair
   carries on average at least 16 source pairs (pf-shell spaces; not sd), it also builds the
   core-pair blocks of the matrix-core products and their slot buffer, which the model keeps:
   n_prot * n_neut * D * 16 doubles for the pn part of two species, and
   C(n, 2) * D * 8 doubles for n nucleons of one species. Setting TRBL_PN_TILES=0 in the
   environment before this call keeps the jump-list and per-element kernels only. */
int trbl_set_hamiltonian(trbl_model* m, const double* spe_p, const double* spe_n, const trbl_tbme* tbme,
                         int64_t n_v);

/* W = H V for a block of nb vectors (App. B, on-the-fly block H.V). V, W: device [D][nb],
   FP64 if precision == TRBL_FP64, FP32 (FP32 accumulation) if TRBL_MIXED. V and W must not alias.
   Products use the model's own work memory: the slot buffer of the core-pair blocks, and the
   work blocks of single-species spaces generated per element. Products and solves of one model
   therefore must not overlap on different streams. With the core-pair blocks, part of the
   product (the proton-proton part, the smaller neutron-sector bins) runs on a second stream that
   the model owns; that work waits for the work already queued on `stream`, and `stream` waits
   for it before the call returns, so the caller sees one stream. */
int trbl_apply(const trbl_model* m, int precision, int nb, const void* V, void* W, void* stream);

/* Lowest n_eig eigenpairs by TRBL (Alg. 4, Sec. 3.4). evals: host n_eig doubles (ascending).
   evecs: optional device [D][n_eig] FP64 Ritz vectors (orthonormal columns). info: optional.
   The QR of each new block is Cholesky QR twice; a block that is numerically rank deficient
   (start block with dependent columns, Krylov space exhausted) is factored column by column
   and its deficient columns are replaced by random vectors orthogonal to the basis
   (info->breakdowns counts them). Device memory: the basis [D][round4(l_m)] in FP64 (or FP32
   with TRBL_MIXED), a packed copy of the current block [D][nb] in the basis precision, one
   FP64 [D][nb] block (plus an FP32 one in mixed mode; the FP64 one also serves as the work
   buffer of restarts that keep more than 208 vectors), small tables; the mixed refinement
   adds two FP64 [D][w] blocks, w = max(1, min(32, 5e8 / D)) columns (at most 8 GB together
   while D <= 5e8).
   Before returning, every returned pair is checked against H itself: the FP64 residual
   ||H x - theta x|| (x formed nb columns at a time when evecs is NULL) must not exceed
   10 * tol * s + 1e-12 * s, s the largest |x^T H x| / x^T x of the returned vectors (mixed mode:
   max(tol, 1e-5) for tol and the refined eigenvalues for s; with TRBL_CONV_RITZ_CHANGE the
   larger of tol * s and the estimate from the projected matrix); these norms go to
   info->resid.
   Returns TRBL_NOT_CONVERGED after max_iter iterations with the current Ritz values (NaN
   beyond the m available when fewer than n_eig exist yet), or when a returned pair fails that
   check (a basis the projected matrix no longer describes).
   Testing aid: with the environment variable TRBL_TEST_CORRUPT_RESTART=1 the first restart
   overwrites half of the first kept Ritz vector, so that the check above must fail. */
int trbl_solve(const trbl_model* m, const trbl_opts* opts, double* evals, void* evecs, trbl_info* info);

/* Gradient of sum_k w_k E_k (Hellmann-Feynman) with respect to every element of the last
   trbl_set_hamiltonian list (grad_v, host n_v) and optionally the proton then neutron
   single-particle energies (grad_spe, host 2*n_orbits, may be NULL).
   evecs: device [D][n_eig] FP64 eigenvectors; NULL = recompute them with trbl_solve(opts).
   TRBL_E_INVALID for single-species spaces that generate their operator per element. */
int trbl_tbme_grad(const trbl_model* m, const trbl_opts* opts, int n_eig, const double* w,
                   const void* evecs, double* grad_v, double* grad_spe);

/* Expectation values <x_c| H |x_c> of the model's Hamiltonian for the n columns of X (device
   [D][n] FP64, the model's basis order), into out (host, n doubles): block H.V (App. B) and
   column products on the device. With H = J^2 written as an interaction (one-body part j(j+1)
   in the single-particle energies, two-body part J(J+1) - ja(ja+1) - jb(jb+1) on diagonal pair
   elements) this gives <J^2> of Ritz vectors. Allocates one [D][min(n,64)] FP64 block. */
int trbl_expect(const trbl_model* m, int n, const void* X, double* out, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
   loops): trbl_expect without any allocation. out is a DEVICE array of n doubles, written on
   `stream` (nothing is copied to the host and nothing waits). The work blocks come from a
   static device buffer of 64 MiB that the library holds on each GPU it runs on until the
   process ends; every call on one GPU shares it, so calls that overlap on one GPU race (order
   them on one stream). The columns go through products of 16, 8, 4, 2 or 1 of them (the widest
   whose D x width FP64 block fits the buffer), whose plans trbl_set_hamiltonian prepares.
   TRBL_E_INVALID when D exceeds the buffer (about 8.3 million states at one column), for
   single-species spaces generated per element, or for bad arguments; TRBL_E_STATE without a
   Hamiltonian. The model's device must be current. */
int trbl_expect_noalloc(const trbl_model* m, int n, const void* X, double* out, void* stream);

/* Particle-hole truncation of Sec. 4.2 (e.g. at most 4 nucleons above the N = 64 subshell gap):
   mask[i] = 1.0 if basis state i has at most max_particles nucleons (protons plus neutrons) in
   the orbits orbit_set[0 .. n_set-1] (host array of orbit indices), else 0.0. mask: device [D]
   FP64, written on `stream`. Errors: TRBL_E_INVALID for a bad orbit index or a negative bound. */
int trbl_occupation_mask(const trbl_model* m, const int* orbit_set, int n_set, int max_particles, double* mask,
                         void* stream);

/* Message of the last failing call on this thread. */
const char* trbl_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TRBL_H */
