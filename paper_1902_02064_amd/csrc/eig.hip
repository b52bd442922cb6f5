// Symmetric eigensolver for the small projected matrix T of TRBL (Alg. 4:
// "diagonalise T^(k)"; restart equations of Sec. 3.4), FP64, in five launches:
//
//   1. Householder reduction to tridiagonal form (A = Q Tri Q^T), reflectors kept
//      (one workgroup: every step depends on the previous one);
//   2. eigenvalues by Sturm-sequence multisection, a group of threads per wanted index,
//      spread over workgroups;
//   3. eigenvectors of Tri by inverse iteration with a pivoted LU of (Tri - lambda I),
//      one thread per vector with its LU in LDS, spread over workgroups;
//   4. Cholesky QR (twice) of the vector block so that vectors of close eigenvalues are
//      orthonormal (Gram tiles and the row solves spread over workgroups, the Cholesky
//      factor on one; skipped when the vectors already are orthonormal);
//   5. back-transformation U = Q Z, one workgroup per block of 16 columns.
// Textbook methods (Householder; Sturm-sequence bisection; inverse iteration),
// written for this library.
#include <cfloat>

#include <hip/hip_cooperative_groups.h>

#include "dense.h"

namespace trbl {

constexpr int EIG_THREADS = 1024;
constexpr int PNB = 8;         // Householder panel width

__device__ static double block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  const int nw = blockDim.x >> 6;
  for (int w = 0; w < nw; w++) s += red[w];
  return s;
}

__device__ static double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ static uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// number of eigenvalues of the tridiagonal (d, e2 = squared off-diagonal) below x
__device__ static int sturm(const double* d, const double* e2, int n, double x, double pivmin) {
  int cnt = 0;
  double q = d[0] - x;
  if (fabs(q) <= pivmin) q = -pivmin;
  if (q < 0.0) cnt++;
  for (int i = 1; i < n; i++) {
    q = d[i] - x - e2[i - 1] / q;
    if (fabs(q) <= pivmin) q = -pivmin;
    if (q < 0.0) cnt++;
  }
  return cnt;
}

constexpr int EIG_BIG = 20 * EIG_NMAX;  // shared work area (doubles)

// Householder reduction to tridiagonal form, unblocked, on ceil(n / TRI_RW) cooperating
// workgroups of 256 threads. Workgroup g holds rows [g TRI_RW, (g+1) TRI_RW) of the current
// matrix in LDS. Step j (reflector H_j = I - 2 v v^T, |v| = 1, acting on rows j+1..n-1):
// every workgroup forms v from row j (which it holds: see below), computes p = A v on its own
// rows and publishes them, and the owner of row j+1 publishes that row as it stands before
// step j; after one grid barrier every workgroup forms w = 2p - 2 (v^T p) v, applies
// A <- A - v w^T - w v^T to its rows and to its copy of row j+1, the next step's row. The
// exchange area alternates between two halves, so one barrier per step suffices: a half is
// rewritten only after every workgroup has passed the barrier that follows its last read.
// Reflector j is kept in row j of A. Output: de[0..n) = d, de[n..2n) = e, de[2n..3n) = e^2,
// de[3n..3n+4) = (lower bound, upper bound, norm bound, pivmin) of the spectrum.
constexpr int TRI_RW = 16;
__global__ __launch_bounds__(256) void tridiag_kernel(const double* __restrict__ T, int ldt, int n,
                                                      double* __restrict__ A, double* __restrict__ de,
                                                      double* __restrict__ xb) {
  extern __shared__ double lds[];
  __shared__ double d[EIG_NMAX], e[EIG_NMAX], e2[EIG_NMAX];
  __shared__ double red[32], wlo[16], whi[16], wnm[16];
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6, nwave = nthr >> 6;
  const int g = blockIdx.x, r0 = g * TRI_RW, nr = min(TRI_RW, n - r0);
  double* Ar = lds;              // nr x n, own rows
  double* v = Ar + TRI_RW * n;   // reflector
  double* w = v + n;             // 2p - 2 (v^T p) v
  double* x = w + n;             // row j of the current matrix
  const int row = tid >> 4, sub = tid & 15;  // p and the update: 16 lanes per own row
  for (int q = tid; q < nr * n; q += nthr) Ar[q] = T[(int64_t)(r0 + q / n) * ldt + q % n];
  for (int c = tid; c < n; c += nthr) x[c] = T[c];
  __syncthreads();
  for (int j = 0; j + 2 < n; j++) {
    double* xh = xb + (int64_t)(j & 1) * 2 * n;  // [0, n): p; [n, 2n): row j+1
    double s = 0.0;
    for (int c = j + 1 + tid; c < n; c += nthr) s += x[c] * x[c];
    const double s2 = block_sum(s, red);
    const double x0 = x[j + 1];
    const double sigma = sqrt(s2);
    if (tid == 0) d[j] = x[j];
    if (sigma == 0.0) {
      for (int c = tid; c < n; c += nthr) v[c] = 0.0;
      if (tid == 0) e[j] = 0.0;
    } else {
      const double alpha = (x0 > 0.0) ? -sigma : sigma;
      const double vn = sqrt(s2 - x0 * x0 + (x0 - alpha) * (x0 - alpha));
      for (int c = tid; c < n; c += nthr) v[c] = c <= j ? 0.0 : (c == j + 1 ? x0 - alpha : x[c]) / vn;
      if (tid == 0) e[j] = alpha;
    }
    __syncthreads();
    if (g == 0)
      for (int c = j + 1 + tid; c < n; c += nthr) A[(int64_t)j * n + c] = v[c];
    const int r = r0 + row;
    if (row < nr && r > j) {
      const double* ar = Ar + row * n;
      double t = 0.0;
      for (int c = j + 1 + sub; c < n; c += 16) t += ar[c] * v[c];
      for (int o = 8; o > 0; o >>= 1) t += __shfl_xor(t, o, 16);
      if (sub == 0) xh[r] = t;
    }
    if (j + 1 >= r0 && j + 1 < r0 + nr)
      for (int c = j + 1 + tid; c < n; c += nthr) xh[n + c] = Ar[(j + 1 - r0) * n + c];
    grid.sync();
    double kp = 0.0;
    for (int c = j + 1 + tid; c < n; c += nthr) {
      const double pc = xh[c];
      w[c] = pc;
      kp += v[c] * pc;
    }
    const double K = block_sum(kp, red);
    for (int c = j + 1 + tid; c < n; c += nthr) w[c] = 2.0 * w[c] - 2.0 * K * v[c];
    __syncthreads();
    if (row < nr && r > j) {
      double* ar = Ar + row * n;
      const double vr = v[r], wr = w[r];
      for (int c = j + 1 + sub; c < n; c += 16) ar[c] -= vr * w[c] + wr * v[c];
    }
    {
      const double vj = v[j + 1], wj = w[j + 1];
      for (int c = j + 1 + tid; c < n; c += nthr) x[c] = xh[n + c] - (vj * w[c] + wj * v[c]);
    }
    __syncthreads();
  }
  // the last two rows: row n-2 is in x; the diagonal of row n-1 comes from its owner
  double* xl = xb + 4 * (int64_t)n;
  if (tid == 0 && n - 1 >= r0 && n - 1 < r0 + nr) xl[0] = Ar[(n - 1 - r0) * n + n - 1];
  grid.sync();
  if (g != 0) return;
  if (tid == 0) {
    if (n >= 2) {
      d[n - 2] = x[n - 2];
      e[n - 2] = x[n - 1];
    }
    d[n - 1] = xl[0];
    e[n - 1] = 0.0;
  }
  __syncthreads();
  for (int i = tid; i < n; i += nthr) e2[i] = e[i] * e[i];
  // Gershgorin interval and a norm bound
  double glo = 1e300, ghi = -1e300, gn = 0.0;
  for (int i = tid; i < n; i += nthr) {
    const double r = fabs(e[i]) + (i > 0 ? fabs(e[i - 1]) : 0.0);
    glo = fmin(glo, d[i] - r);
    ghi = fmax(ghi, d[i] + r);
    gn = fmax(gn, fabs(d[i]) + r);
  }
  for (int o = 32; o > 0; o >>= 1) {
    glo = fmin(glo, __shfl_down(glo, o, 64));
    ghi = fmax(ghi, __shfl_down(ghi, o, 64));
    gn = fmax(gn, __shfl_down(gn, o, 64));
  }
  if (lane == 0) {
    wlo[wave] = glo;
    whi[wave] = ghi;
    wnm[wave] = gn;
  }
  __syncthreads();
  glo = 1e300;
  ghi = -1e300;
  gn = 0.0;
  for (int w = 0; w < nwave; w++) {
    glo = fmin(glo, wlo[w]);
    ghi = fmax(ghi, whi[w]);
    gn = fmax(gn, wnm[w]);
  }
  const double tnorm = fmax(gn, DBL_MIN);
  const double pivmin = DBL_MIN * fmax(1.0, tnorm * tnorm);
  glo -= 2.0 * DBL_EPSILON * tnorm * n + pivmin;
  ghi += 2.0 * DBL_EPSILON * tnorm * n + pivmin;
  for (int i = tid; i < n; i += nthr) {
    de[i] = d[i];
    de[n + i] = e[i];
    de[2 * n + i] = e2[i];
  }
  if (tid == 0) {
    de[3 * n] = glo;
    de[3 * n + 1] = ghi;
    de[3 * n + 2] = tnorm;
    de[3 * n + 3] = pivmin;
  }
}


// eigenvalues by multisection: a group of BIS_TPE threads refines one eigenvalue (the nvec
// lowest and the largest); each round its threads take Sturm counts at BIS_TPE interior points
// of the group's interval, which shrinks by a factor BIS_TPE + 1. Launch: 256 threads per
// workgroup, ceil((nvec + 1) * BIS_TPE / 256) workgroups.
constexpr int BIS_TPE = 32;
__global__ __launch_bounds__(256) void bisect_kernel(const double* __restrict__ de, int n, int nvec,
                                                     double* __restrict__ theta) {
  __shared__ double d[EIG_NMAX], e2[EIG_NMAX];
  __shared__ double sx[256];
  __shared__ int scnt[256];
  const int tid = threadIdx.x, nthr = blockDim.x;
  for (int i = tid; i < n; i += nthr) {
    d[i] = de[i];
    e2[i] = de[2 * n + i];
  }
  double glo = de[3 * n], ghi = de[3 * n + 1];
  const double pivmin = de[3 * n + 3];
  __syncthreads();
  {
    const int tpe = BIS_TPE;
    const int q = blockIdx.x * (nthr / tpe) + tid / tpe, sub = tid % tpe;
    const int want = q < nvec ? q : ((q == nvec && nvec < n) ? n - 1 : -1);
    double lo = glo, hi = ghi;
    const int rounds = (int)ceil(64.0 / log2((double)tpe + 1.0)) + 1;
    for (int rd = 0; rd < rounds; rd++) {
      const bool live =
          want >= 0 && !(hi - lo <= 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)) + 2.0 * pivmin);
      double x = lo;
      int cnt = -1;
      if (live) {
        x = lo + (hi - lo) * (double)(sub + 1) / (double)(tpe + 1);
        cnt = sturm(d, e2, n, x, pivmin);
      }
      sx[tid] = x;
      scnt[tid] = cnt;
      __syncthreads();
      if (live) {
        double nlo = lo, nhi = hi;
        for (int t = 0; t < tpe; t++) {
          const double xt = sx[(tid / tpe) * tpe + t];
          if (scnt[(tid / tpe) * tpe + t] > want) nhi = fmin(nhi, xt);
          else nlo = fmax(nlo, xt);
        }
        lo = nlo;
        hi = nhi;
      }
      __syncthreads();
    }
    if (want >= 0 && sub == 0) theta[want] = 0.5 * (lo + hi);
  }
}

// inverse iteration, one thread per wanted vector. The pivoted LU of (Tri - lambda I) is
// computed with the running pivot row kept in registers and written out once to LDS; the
// solves stream through it. Column j of Z (row-major, stride nvec) receives vector j.
// Launch: ceil(nvec / INV_VPW) workgroups of 64 threads, 2 n + INV_VPW (6 n + 4) doubles of LDS.
constexpr int INV_VPW = 4;
__global__ __launch_bounds__(64) void inviter_kernel(const double* __restrict__ de, const double* __restrict__ theta,
                                                     int n, int nvec, double* __restrict__ Z) {
  extern __shared__ double lds[];
  const int tid = threadIdx.x;
  double* d = lds;
  double* e = lds + n;
  for (int i = tid; i < n; i += blockDim.x) {
    d[i] = de[i];
    e[i] = de[n + i];
  }
  const double tnorm = de[3 * n + 2];
  __syncthreads();
  {
    const int jl = tid;
    const int j = blockIdx.x * INV_VPW + jl;
    if (jl >= INV_VPW || j >= nvec) return;
    double* dl = lds + 2 * n + (int64_t)jl * (6 * n + 4);  // padded against bank conflicts
    double* dd = dl + n;
    double* du = dd + n;
    double* du2 = du + n;
    double* pv = du2 + n;
    double* zl = pv + n;
#define AT(p, i) (p)[(i)]
    const double lm = theta[j];
    const double tiny = DBL_EPSILON * tnorm;
    // running values of the current pivot row: a = dd[i], u1 = du[i]
    double a = d[0] - lm, u1 = e[0];
    for (int i = 0; i + 1 < n; i++) {
      const double b = e[i];                  // sub-diagonal below the pivot
      const double dnext = d[i + 1] - lm, enext = (i + 2 < n) ? e[i + 1] : 0.0;
      double piv, sup, sup2, mult, na, nu1;
      bool sw;
      if (fabs(a) >= fabs(b)) {
        sw = false;
        piv = a;
        sup = u1;
        sup2 = 0.0;
        mult = (a != 0.0) ? b / a : 0.0;
        na = dnext - mult * u1;
        nu1 = enext;
      } else {
        sw = true;
        piv = b;
        sup = dnext;
        sup2 = enext;
        mult = a / b;
        na = u1 - mult * dnext;
        nu1 = -mult * enext;
      }
      if (fabs(piv) < tiny) piv = (piv < 0.0) ? -tiny : tiny;
      AT(dd, i) = piv;
      AT(du, i) = sup;
      AT(du2, i) = sup2;
      AT(dl, i) = mult;
      AT(pv, i) = sw ? 1.0 : 0.0;
      a = na;
      u1 = nu1;
    }
    if (fabs(a) < tiny) a = (a < 0.0) ? -tiny : tiny;
    AT(dd, n - 1) = a;
    AT(du, n - 1) = 0.0;
    AT(du2, n - 1) = 0.0;
    double* z = zl;
    uint64_t h = mix64(0x5D0C5EEDull + (uint64_t)j * 1315423911ull);
    for (int i = 0; i < n; i++) {
      h = mix64(h + i);
      AT(z, i) = ((double)(h >> 11) * (1.0 / 9007199254740992.0)) - 0.5;
    }
    for (int it = 0; it < 3; it++) {
      // forward: row interchanges and L, with the two live entries in registers
      double zc = AT(z, 0);
      for (int i = 0; i + 1 < n; i++) {
        double zn = AT(z, i + 1);
        if (AT(pv, i) != 0.0) {
          const double t = zc;
          zc = zn;
          zn = t;
        }
        AT(z, i) = zc;
        zc = zn - AT(dl, i) * zc;
      }
      AT(z, n - 1) = zc;
      // backward: U, carrying z[i+1], z[i+2]
      double z1 = AT(z, n - 1) / AT(dd, n - 1), z2 = 0.0;
      AT(z, n - 1) = z1;
      for (int i = n - 2; i >= 0; i--) {
        const double zi = (AT(z, i) - AT(du, i) * z1 - AT(du2, i) * z2) / AT(dd, i);
        AT(z, i) = zi;
        z2 = z1;
        z1 = zi;
      }
      double nr = 0.0;
      for (int i = 0; i < n; i++) nr += AT(z, i) * AT(z, i);
      nr = 1.0 / sqrt(nr);
      for (int i = 0; i < n; i++) AT(z, i) *= nr;
    }
#undef AT
    for (int i = 0; i < n; i++) Z[(int64_t)i * nvec + j] = zl[i];
  }
}

// Cholesky QR, twice, of Z (n x nvec, row-major), when orthonormal vectors are needed
// (restarts, final vectors). Each pass: G = Z^T Z (gram_kernel); if max |G - I| <= 64 eps the
// vectors are already orthonormal to working accuracy (well separated eigenvalues) and the
// flag `done` ends the procedure; otherwise the upper Cholesky factor R of G (chol_g_kernel)
// and Z <- Z R^-1 (rsolve_kernel). Every kernel returns at once when `done` is set.
typedef double d4e __attribute__((ext_vector_type(4)));
__device__ __forceinline__ d4e mfma_f64(double a, double b, d4e c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__global__ void clear_flag_kernel(int* f) { *f = 0; }

// upper 16 x 16 tiles of G = Z^T Z, one wavefront per tile (MFMA f64 16x16x4 over 4 rows of Z)
__global__ __launch_bounds__(64) void gram_kernel(const double* __restrict__ Z, int n, int nvec,
                                                  double* __restrict__ G, const int* done) {
  if (*done) return;
  const int nt = (nvec + 15) / 16;
  int t = blockIdx.x, rt = 0;
  while (t >= nt - rt) {
    t -= nt - rt;
    rt++;
  }
  const int ct = rt + t;
  const int li = threadIdx.x & 15, lk = threadIdx.x >> 4;
  const int ca = rt * 16 + li, cb = ct * 16 + li;
  d4e acc = {0, 0, 0, 0};
  for (int i0 = 0; i0 < n; i0 += 4) {
    const int i = i0 + lk;
    const double x = (i < n && ca < nvec) ? Z[(int64_t)i * nvec + ca] : 0.0;
    const double y = (i < n && cb < nvec) ? Z[(int64_t)i * nvec + cb] : 0.0;
    acc = mfma_f64(x, y, acc);
  }
#pragma unroll
  for (int v = 0; v < 4; v++) {
    const int r = rt * 16 + lk + 4 * v;
    if (r < nvec && cb < nvec && cb >= r) G[(int64_t)r * nvec + cb] = acc[v];
  }
}

// orthonormality test, then the upper Cholesky G = R^T R in place (row k finalised at step k)
__global__ __launch_bounds__(EIG_THREADS) void chol_g_kernel(int nvec, double* __restrict__ G, int* done) {
  __shared__ double red[32];
  if (*done) return;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6, nwave = nthr >> 6;
  double off = 0.0;
  for (int r = wave; r < nvec; r += nwave)
    for (int c = r + lane; c < nvec; c += 64) off = fmax(off, fabs(G[(int64_t)r * nvec + c] - (r == c ? 1.0 : 0.0)));
  for (int o = 32; o > 0; o >>= 1) off = fmax(off, __shfl_xor(off, o, 64));
  if (lane == 0) red[wave] = off;
  __syncthreads();
  off = 0.0;
  for (int w = 0; w < nwave; w++) off = fmax(off, red[w]);
  if (off <= 64.0 * DBL_EPSILON) {
    if (tid == 0) *done = 1;
    return;
  }
  for (int k = 0; k < nvec; k++) {
    const double rkk = sqrt(fmax(G[(int64_t)k * nvec + k], 1e-300));
    __syncthreads();
    for (int c = k + 1 + tid; c < nvec; c += nthr) G[(int64_t)k * nvec + c] /= rkk;
    if (tid == 0) G[(int64_t)k * nvec + k] = rkk;
    __syncthreads();
    for (int r = k + 1 + wave; r < nvec; r += nwave) {
      const double gkr = G[(int64_t)k * nvec + r];
      for (int c = r + lane; c < nvec; c += 64) G[(int64_t)r * nvec + c] -= gkr * G[(int64_t)k * nvec + c];
    }
    __syncthreads();
  }
}

// Z <- Z R^-1, 16 rows per workgroup: 16 lanes share a row (staged in LDS) and solve x R = z
// column by column, each dot split over the 16 lanes
__global__ __launch_bounds__(256) void rsolve_kernel(int n, int nvec, double* __restrict__ Z,
                                                     const double* __restrict__ G, const int* done) {
  __shared__ double zs[16 * EIG_NMAX];
  if (*done) return;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int i0 = blockIdx.x * 16, rr = min(16, n - i0);
  for (int q = tid; q < rr * nvec; q += nthr) zs[q] = Z[(int64_t)i0 * nvec + q];
  __syncthreads();
  const int row = tid >> 4, sub = tid & 15;
  if (row < rr) {
    double* zr = zs + row * nvec;
    for (int c = 0; c < nvec; c++) {
      double s = 0.0;
      for (int r = sub; r < c; r += 16) s += zr[r] * G[(int64_t)r * nvec + c];
      for (int o = 8; o > 0; o >>= 1) s += __shfl_xor(s, o, 16);
      const double val = (zr[c] - s) / G[(int64_t)c * nvec + c];
      __builtin_amdgcn_wave_barrier();
      if (sub == 0) zr[c] = val;
      __builtin_amdgcn_wave_barrier();
    }
  }
  __syncthreads();
  for (int q = tid; q < rr * nvec; q += nthr) Z[(int64_t)i0 * nvec + q] = zs[q];
}

// back-transformation U = H_0 H_1 ... H_{n-3} Z (reflectors applied last to first): one
// workgroup per block of 16 columns, held in LDS, one wave per column; nr reflectors at a
// time are staged in LDS (zero-padded to full length) between barriers.
__global__ __launch_bounds__(EIG_THREADS) void backtr_kernel(const double* __restrict__ A, int n, int nvec,
                                                             const double* __restrict__ Z, double* __restrict__ U,
                                                             int ldu) {
  __shared__ double big[EIG_BIG];
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6;
  {
    double* zs = big;
    double* vb = big + 16 * n;
    const int nr = max(1, min(16, (EIG_BIG - 16 * n) / n));
    {
      const int cb = 16 * blockIdx.x;
      const int ncol = min(16, nvec - cb);
      for (int q = tid; q < n * ncol; q += nthr) {
        const int i = q / ncol, c = q - (q / ncol) * ncol;
        zs[c * n + i] = Z[(int64_t)i * nvec + cb + c];
      }
      for (int k0 = n - 3; k0 >= 0; k0 -= nr) {
        __syncthreads();
        for (int q = tid; q < nr * n; q += nthr) {
          const int t = q / n, i = q - (q / n) * n, k = k0 - t;
          vb[q] = (k >= 0 && i > k) ? A[(int64_t)k * n + i] : 0.0;
        }
        __syncthreads();
        if (wave < ncol) {
          double* z = zs + wave * n;
          for (int t = 0; t < nr && k0 - t >= 0; t++) {
            const int k = k0 - t;
            const double* v = vb + t * n;
            double sdot = 0.0;
            for (int i = k + 1 + lane; i < n; i += 64) sdot += v[i] * z[i];
            sdot = 2.0 * wave_sum(sdot);
            for (int i = k + 1 + lane; i < n; i += 64) z[i] -= sdot * v[i];
          }
        }
      }
      __syncthreads();
      for (int q = tid; q < n * ncol; q += nthr) {
        const int i = q / ncol, c = q - (q / ncol) * ncol;
        U[(int64_t)i * ldu + cb + c] = zs[c * n + i];
      }
      __syncthreads();
    }
  }
}

void symeig(const double* T, int ldt, int n, int nvec, double* theta, double* U, int ldu, EigWork& w, bool orth,
            hipStream_t st) {
  TRBL_REQUIRE(n >= 1 && n <= EIG_NMAX && nvec >= 1 && nvec <= n, TRBL_E_INVALID, "eigensolver size out of range");
  w.a.alloc((size_t)n * n * sizeof(double));
  w.z.alloc((size_t)n * nvec * sizeof(double));
  w.lu.alloc((size_t)nvec * nvec * sizeof(double));
  w.aux.alloc((size_t)(3 * n + 4) * sizeof(double));
  w.xb.alloc((size_t)(4 * n + 8) * sizeof(double));
  w.flag.alloc(sizeof(int));
  double* de = w.aux.as<double>();
  {
    double* A = w.a.as<double>();
    double* xb = w.xb.as<double>();
    void* args[] = {(void*)&T, (void*)&ldt, (void*)&n, (void*)&A, (void*)&de, (void*)&xb};
    const size_t shm = (size_t)(TRI_RW + 3) * n * sizeof(double);
    TRBL_HIP(hipLaunchCooperativeKernel((const void*)tridiag_kernel, dim3((n + TRI_RW - 1) / TRI_RW), dim3(256), args,
                                        (unsigned)shm, st));
  }
  const int nwant = nvec < n ? nvec + 1 : nvec;
  hipLaunchKernelGGL(bisect_kernel, dim3((nwant * BIS_TPE + 255) / 256), dim3(256), 0, st, de, n, nvec, theta);
  hipLaunchKernelGGL(inviter_kernel, dim3((nvec + INV_VPW - 1) / INV_VPW), dim3(64),
                     (size_t)(2 * n + INV_VPW * (6 * n + 4)) * sizeof(double), st, de, theta, n, nvec,
                     w.z.as<double>());
  if (orth && nvec > 1) {
    int* done = w.flag.as<int>();
    const int nt = (nvec + 15) / 16;
    hipLaunchKernelGGL(clear_flag_kernel, dim3(1), dim3(1), 0, st, done);
    for (int pass = 0; pass < 2; pass++) {
      hipLaunchKernelGGL(gram_kernel, dim3(nt * (nt + 1) / 2), dim3(64), 0, st, w.z.as<double>(), n, nvec,
                         w.lu.as<double>(), done);
      hipLaunchKernelGGL(chol_g_kernel, dim3(1), dim3(EIG_THREADS), 0, st, nvec, w.lu.as<double>(), done);
      hipLaunchKernelGGL(rsolve_kernel, dim3((n + 15) / 16), dim3(256), 0, st, n, nvec, w.z.as<double>(),
                         w.lu.as<double>(), done);
    }
  }
  hipLaunchKernelGGL(backtr_kernel, dim3((nvec + 15) / 16), dim3(EIG_THREADS), 0, st, w.a.as<double>(), n, nvec,
                     w.z.as<double>(), U, ldu);
  TRBL_HIP(hipGetLastError());
}

}  // namespace trbl

namespace trbl {

// M = L^-1 S L^-T with G = L L^T (one workgroup, n <= 1024)
__global__ __launch_bounds__(1024) void gen_reduce_kernel(const double* __restrict__ S, const double* __restrict__ G,
                                                          int n, double* __restrict__ M, double* __restrict__ L,
                                                          double* __restrict__ Li, int* status) {
  const int tid = threadIdx.x, nthr = blockDim.x;
  __shared__ int bad;
  if (tid == 0) bad = 0;
  for (int64_t q = tid; q < (int64_t)n * n; q += nthr) {
    const int i = (int)(q / n), j = (int)(q % n);
    L[q] = (j <= i) ? 0.5 * (G[q] + G[(int64_t)j * n + i]) : 0.0;
  }
  __syncthreads();
  // left-looking Cholesky, lower triangular L
  for (int k = 0; k < n; k++) {
    if (tid == 0) {
      double p = L[(int64_t)k * n + k];
      for (int q = 0; q < k; q++) p -= L[(int64_t)k * n + q] * L[(int64_t)k * n + q];
      if (!(p > 0.0)) {
        bad = 1;
        p = 1e-300;
      }
      L[(int64_t)k * n + k] = sqrt(p);
    }
    __syncthreads();
    const double lkk = L[(int64_t)k * n + k];
    for (int i = k + 1 + tid; i < n; i += nthr) {
      double s = L[(int64_t)i * n + k];
      for (int q = 0; q < k; q++) s -= L[(int64_t)i * n + q] * L[(int64_t)k * n + q];
      L[(int64_t)i * n + k] = s / lkk;
    }
    __syncthreads();
  }
  // Li = L^-1 (lower), one thread per column
  for (int j = tid; j < n; j += nthr) {
    for (int i = 0; i < n; i++) Li[(int64_t)i * n + j] = 0.0;
    Li[(int64_t)j * n + j] = 1.0 / L[(int64_t)j * n + j];
    for (int i = j + 1; i < n; i++) {
      double s = 0.0;
      for (int q = j; q < i; q++) s += L[(int64_t)i * n + q] * Li[(int64_t)q * n + j];
      Li[(int64_t)i * n + j] = -s / L[(int64_t)i * n + i];
    }
  }
  __syncthreads();
  // M = Li S Li^T, via P = Li S (stored in L) then M = P Li^T
  for (int64_t q = tid; q < (int64_t)n * n; q += nthr) {
    const int i = (int)(q / n), j = (int)(q % n);
    double s = 0.0;
    for (int t = 0; t <= i; t++) s += Li[(int64_t)i * n + t] * 0.5 * (S[(int64_t)t * n + j] + S[(int64_t)j * n + t]);
    L[q] = s;
  }
  __syncthreads();
  for (int64_t q = tid; q < (int64_t)n * n; q += nthr) {
    const int i = (int)(q / n), j = (int)(q % n);
    double s = 0.0;
    for (int t = 0; t <= j; t++) s += L[(int64_t)i * n + t] * Li[(int64_t)j * n + t];
    M[q] = s;
  }
  __syncthreads();
  for (int64_t q = tid; q < (int64_t)n * n; q += nthr) {
    const int i = (int)(q / n), j = (int)(q % n);
    if (j < i) M[q] = M[(int64_t)j * n + i] = 0.5 * (M[q] + M[(int64_t)j * n + i]);
  }
  if (tid == 0) status[0] = bad;
}

__global__ void gen_back_kernel(const double* Li, const double* Yp, int ldp, int n, int nv, double* Y, int ldy) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= (int64_t)n * nv) return;
  const int i = (int)(q / nv), j = (int)(q % nv);
  double s = 0.0;
  for (int t = i; t < n; t++) s += Li[(int64_t)t * n + i] * Yp[(int64_t)t * ldp + j];  // (L^-T)_{it} = Li_{ti}
  Y[(int64_t)i * ldy + j] = s;
}

__global__ void reduce_partials_kernel_eig(const double* part, int G, int len, double* out) {
  const int k = threadIdx.x;
  if (k >= len) return;
  double s = 0.0;
  for (int g = 0; g < G; g++) s += part[(int64_t)g * len + k];
  out[k] = s;
}

__global__ void resid_cols_kernel(const double* W, int64_t ldw, const double* X, int64_t ldx, const double* theta,
                                  int ncol, int64_t D, int64_t rows_per, double* part) {
  const int c = threadIdx.x % 64;
  const int rsub = threadIdx.x / 64;
  __shared__ double acc[4][64];
  double s = 0.0;
  const int64_t r0 = blockIdx.x * rows_per, r1 = min(D, r0 + rows_per);
  if (c < ncol)
    for (int64_t r = r0 + rsub; r < r1; r += 4) {
      const double x = W[r * ldw + c] - theta[c] * X[r * ldx + c];
      s += x * x;
    }
  acc[rsub][c] = s;
  __syncthreads();
  if (rsub == 0 && c < ncol) part[(int64_t)blockIdx.x * ncol + c] = acc[0][c] + acc[1][c] + acc[2][c] + acc[3][c];
}

__global__ void dot_cols_kernel(const double* W, int64_t ldw, const double* X, int64_t ldx, int ncol, int64_t D,
                                int64_t rows_per, double* part) {
  const int c = threadIdx.x % 64;
  const int rsub = threadIdx.x / 64;
  __shared__ double acc[4][64];
  double s = 0.0;
  const int64_t r0 = blockIdx.x * rows_per, r1 = min(D, r0 + rows_per);
  if (c < ncol)
    for (int64_t r = r0 + rsub; r < r1; r += 4) s += W[r * ldw + c] * X[r * ldx + c];
  acc[rsub][c] = s;
  __syncthreads();
  if (rsub == 0 && c < ncol) part[(int64_t)blockIdx.x * ncol + c] = acc[0][c] + acc[1][c] + acc[2][c] + acc[3][c];
}

void gen_reduce(const double* S, const double* G, int n, double* M, double* Linv, int* status, hipStream_t st) {
  static thread_local DevBuf Lb;
  Lb.alloc((size_t)n * n * sizeof(double));
  hipLaunchKernelGGL(gen_reduce_kernel, dim3(1), dim3(1024), 0, st, S, G, n, M, Lb.as<double>(), Linv, status);
  TRBL_HIP(hipGetLastError());
}

void gen_back(const double* Linv, const double* Yp, int ldp, int n, int nv, double* Y, int ldy, hipStream_t st) {
  const int64_t tot = (int64_t)n * nv;
  hipLaunchKernelGGL(gen_back_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, Linv, Yp, ldp, n, nv, Y,
                     ldy);
  TRBL_HIP(hipGetLastError());
}

void resid_cols(const double* W, int64_t ldw, const double* X, int64_t ldx, const double* theta, int ncol, int64_t D,
                double* out, Scratch& s, hipStream_t st) {
  TRBL_REQUIRE(ncol <= 64, TRBL_E_INVALID, "resid_cols: at most 64 columns per call");
  int G = (int)std::min<int64_t>(1024, std::max<int64_t>(1, D / 1024));
  const int64_t rows_per = (D + G - 1) / G;
  G = (int)((D + rows_per - 1) / rows_per);
  double* part = s.partials((size_t)G * ncol);
  hipLaunchKernelGGL(resid_cols_kernel, dim3(G), dim3(256), 0, st, W, ldw, X, ldx, theta, ncol, D, rows_per, part);
  hipLaunchKernelGGL(reduce_partials_kernel_eig, dim3(1), dim3(64), 0, st, part, G, ncol, out);
  TRBL_HIP(hipGetLastError());
}

int dot_cols_parts(int64_t D) { return (int)std::min<int64_t>(1024, std::max<int64_t>(1, D / 1024)); }

void dot_cols(const double* W, int64_t ldw, const double* X, int64_t ldx, int ncol, int64_t D, double* part,
              double* out, hipStream_t st) {
  TRBL_REQUIRE(ncol >= 1 && ncol <= 64, TRBL_E_INVALID, "dot_cols: 1 to 64 columns per call");
  int G = dot_cols_parts(D);
  const int64_t rows_per = (D + G - 1) / G;
  G = (int)((D + rows_per - 1) / rows_per);
  hipLaunchKernelGGL(dot_cols_kernel, dim3(G), dim3(256), 0, st, W, ldw, X, ldx, ncol, D, rows_per, part);
  hipLaunchKernelGGL(reduce_partials_kernel_eig, dim3(1), dim3(64), 0, st, part, G, ncol, out);
  TRBL_HIP(hipGetLastError());
}

}  // namespace trbl
