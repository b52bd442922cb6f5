// Dense block kernels of TRBL (Alg. 4): projections V^T W, block Gram-Schmidt
// updates W -= V C, Cholesky QR of the new block, and the restart combination
// v_k := sum_j v_j U_jk (Sec. 3.4). All arithmetic is FP64; stored vectors may
// be FP32 (mixed precision) and are widened on load.
//
// Matrix-core use: v_mfma_f64_16x16x4f64. Operand layout (one double per lane):
//   A (16 x 4):  lane l holds A[l % 16][l / 16]
//   B (4 x 16):  lane l holds B[l / 16][l % 16]
//   D (16 x 16): lane l, register v holds D[l / 16 + 4 * v][l % 16], v = 0..3 (measured on gfx950)
// In row-streaming products the k index of a 16-wide chunk is permuted so each
// lane loads 4 consecutive values of one row (k = k0 + 4 * (l / 16) + t for
// step t): the sum over k is unchanged and the loads are 128-byte coalesced.
#include "dense.h"

namespace trbl {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <class T>
__device__ __forceinline__ double ld(const T* p) {
  return (double)(*p);
}

// four consecutive values of a row in their own type; masked beyond `valid`
template <class T>
__device__ __forceinline__ void ld4raw(const T* p, int valid, T out[4]) {
  if (valid >= 4) {
    if constexpr (sizeof(T) == 8) {
      const double2* q = reinterpret_cast<const double2*>(p);
      double2 x = q[0], y = q[1];
      out[0] = x.x; out[1] = x.y; out[2] = y.x; out[3] = y.y;
    } else {
      float4 x = *reinterpret_cast<const float4*>(p);
      out[0] = x.x; out[1] = x.y; out[2] = x.z; out[3] = x.w;
    }
  } else {
#pragma unroll
    for (int t = 0; t < 4; t++) out[t] = (t < valid) ? p[t] : T(0);
  }
}

// four consecutive values of a row, widened; masked beyond `valid`
template <class T>
__device__ __forceinline__ void ld4(const T* p, int valid, double out[4]) {
  if (valid >= 4) {
    if constexpr (sizeof(T) == 8) {
      const double2* q = reinterpret_cast<const double2*>(p);
      double2 x = q[0], y = q[1];
      out[0] = x.x; out[1] = x.y; out[2] = y.x; out[3] = y.y;
    } else {
      float4 x = *reinterpret_cast<const float4*>(p);
      out[0] = x.x; out[1] = x.y; out[2] = x.z; out[3] = x.w;
    }
  } else {
#pragma unroll
    for (int t = 0; t < 4; t++) out[t] = (t < valid) ? (double)p[t] : 0.0;
  }
}

// ------------------------------------------------------------------ C = A^T B (partial per workgroup)
// A: [D][lda] (m columns used), B: [D][ldb] (nb columns). part[g] is m x nb row-major.
// Workgroup (x, y) covers a row chunk and the column chunk [64 NP y, 64 NP (y + 1)) of A; each
// wave takes row quads of the chunk. In a 64-column panel, lane l loads 4 consecutive
// values A[r][c0 + 4 (l % 16) + t] of row r = 4-row quad + l / 16 (32 bytes), and value t
// feeds MFMA t, whose output row i then stands for column c0 + 4 i + t.
template <class TA, class TB, int NP, int MAXC>
__global__ __launch_bounds__(256) void tn_partial_kernel(const TA* __restrict__ A, int64_t lda, int m,
                                                         const TB* __restrict__ B, int64_t ldb, int nb, int64_t D,
                                                         int64_t rows_per, double* __restrict__ part) {
  constexpr int WAVES = 4;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ct = (nb + 15) >> 4;
  const int cbase = blockIdx.y * 64 * NP;
  d4 acc[NP][4][MAXC];
#pragma unroll
  for (int p = 0; p < NP; p++)
#pragma unroll
    for (int t = 0; t < 4; t++)
#pragma unroll
      for (int q = 0; q < MAXC; q++) acc[p][t][q] = d4{0, 0, 0, 0};
  const int64_t r0 = (int64_t)blockIdx.x * rows_per;
  const int64_t r1 = min(D, r0 + rows_per);
  const int li = lane & 15, lk = lane >> 4;
  for (int64_t r = r0 + 4 * wave; r < r1; r += 4 * WAVES) {
    const int64_t rr = r + lk;
    const bool rok = rr < r1;
    double bop[MAXC];
#pragma unroll
    for (int q = 0; q < MAXC; q++) {
      const int c = q * 16 + li;
      bop[q] = (q < ct && rok && c < nb) ? ld(B + rr * ldb + c) : 0.0;
    }
#pragma unroll
    for (int p = 0; p < NP; p++) {
      const int c0 = cbase + 64 * p + 4 * li;
      double a4[4];
      if (rok && c0 < m) ld4(A + rr * lda + c0, m - c0, a4);
      else a4[0] = a4[1] = a4[2] = a4[3] = 0.0;
#pragma unroll
      for (int t = 0; t < 4; t++)
#pragma unroll
        for (int q = 0; q < MAXC; q++)
          if (q < ct) acc[p][t][q] = mfma(a4[t], bop[q], acc[p][t][q]);
    }
  }
  // combine the waves' sums in LDS (one wave after the other), then write the chunk's partial
  constexpr int NBS = 16 * MAXC;
  __shared__ double red[64 * NP * NBS];
  const int ncol = min(64 * NP, m - cbase);
  for (int e = threadIdx.x; e < 64 * NP * NBS; e += blockDim.x) red[e] = 0.0;
  for (int w = 0; w < WAVES; w++) {
    __syncthreads();
    if (wave != w) continue;
#pragma unroll
    for (int p = 0; p < NP; p++)
#pragma unroll
      for (int t = 0; t < 4; t++)
#pragma unroll
        for (int q = 0; q < MAXC; q++) {
          if (q >= ct) continue;
#pragma unroll
          for (int v = 0; v < 4; v++) {
            const int col = 64 * p + 4 * (lk + 4 * v) + t, c = q * 16 + li;
            if (col < ncol && c < nb) red[col * NBS + c] += acc[p][t][q][v];
          }
        }
  }
  __syncthreads();
  double* out = part + (int64_t)blockIdx.x * m * nb + (int64_t)cbase * nb;
  for (int e = threadIdx.x; e < ncol * nb; e += blockDim.x) out[e] = red[(e / nb) * NBS + e % nb];
}

// out[k] = sum_g part[g * len + k]: 16 outputs per block, 16 threads share the G terms of each
// (fixed summation order, so results are reproducible)
__global__ __launch_bounds__(256) void reduce_partials_kernel(const double* __restrict__ part, int G, int64_t len,
                                                              double* __restrict__ out) {
  __shared__ double red[16][17];
  const int kx = threadIdx.x & 15, gy = threadIdx.x >> 4;
  const int64_t k = (int64_t)blockIdx.x * 16 + kx;
  double s = 0.0;
  if (k < len)
#pragma unroll 8
    for (int g = gy; g < G; g += 16) s += part[(int64_t)g * len + k];
  red[gy][kx] = s;
  __syncthreads();
  if (gy == 0 && k < len) {
    double t = 0.0;
    for (int j = 0; j < 16; j++) t += red[j][kx];
    out[k] = t;
  }
}

// ------------------------------------------------------------------ Bout = Bin - A C (+ fused partial product)
// (Bin == nullptr: Bout = A C.)
// mode 0: update only; mode 1: also part[g] += A^T Bout (m x nb); mode 2: also part[g] += Bout^T Bout (nb x nb).
// C (m x nb, FP64) is staged in LDS, padded to 16-multiples with zeros.
// Bout may be FP32 (the mixed-precision block kept in the basis array): the fused products then
// use the stored (rounded) values.
template <class TA, class TI, class TO, int WAVES, int MAXI, int MAXC>
__global__ __launch_bounds__(WAVES * 64) void update_kernel(const TA* __restrict__ A, int64_t lda, int m,
                                                     const double* __restrict__ C, const TI* Bin, int64_t ldi,
                                                     TO* Bout, int64_t ldo, int nb, int64_t D, int mode,
                                                     double* __restrict__ part, TO* Bout2, int64_t ldo2) {
  constexpr int ROWS = WAVES * 16;
  extern __shared__ double lds[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int mt = (m + 15) >> 4, ct = (nb + 15) >> 4;
  const int mp = mt * 16, nbp = ct * 16;
  double* Cs = lds;                 // mp x nbp
  double* Wt = lds + mp * nbp;      // ROWS x nbp
  for (int e = threadIdx.x; e < mp * nbp; e += blockDim.x) {
    const int k = e / nbp, c = e % nbp;
    Cs[e] = (k < m && c < nb) ? C[k * nb + c] : 0.0;
  }
  __syncthreads();
  const int li = lane & 15, lk = lane >> 4;
  const int npan = (m + 63) >> 6;  // 64-column panels of A (mode 1: panel p belongs to wave p % WAVES)
  d4 pacc[MAXI][4][MAXC];          // mode 1: [panel slot][t][column tile]; mode 2: [0][qi][qj]
#pragma unroll
  for (int i = 0; i < MAXI; i++)
#pragma unroll
    for (int t = 0; t < 4; t++)
#pragma unroll
      for (int q = 0; q < MAXC; q++) pacc[i][t][q] = d4{0, 0, 0, 0};
  const int64_t ntiles = (D + ROWS - 1) / ROWS;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t rbase = tile * ROWS;
    // ---- phase 1: each wave updates its 16 rows
    const int64_t rw = rbase + wave * 16;
    d4 acc[MAXC];
#pragma unroll
    for (int q = 0; q < MAXC; q++) acc[q] = d4{0, 0, 0, 0};
    const int64_t ra = rw + li;  // row this lane loads for the A operand
    for (int k0 = 0; k0 < m; k0 += 16) {
      const int kk = k0 + 4 * lk;
      double a4[4];
      if (ra < D) ld4(A + ra * lda + kk, m - kk, a4);
      else a4[0] = a4[1] = a4[2] = a4[3] = 0.0;
#pragma unroll
      for (int t = 0; t < 4; t++) {
#pragma unroll
        for (int q = 0; q < MAXC; q++)
          if (q < ct) acc[q] = mfma(a4[t], Cs[(kk + t) * nbp + q * 16 + li], acc[q]);
      }
    }
#pragma unroll
    for (int q = 0; q < MAXC; q++) {
      if (q >= ct) continue;
#pragma unroll
      for (int v = 0; v < 4; v++) {
        const int rl = wave * 16 + lk + 4 * v;
        const int64_t r = rbase + rl;
        const int c = q * 16 + li;
        double val = 0.0;
        if (r < D && c < nb) {
          const TO out = (TO)(Bin ? ld(Bin + r * ldi + c) - acc[q][v] : acc[q][v]);
          Bout[r * ldo + c] = out;
          if (Bout2) Bout2[r * ldo2 + c] = out;
          val = (double)out;
        }
        Wt[rl * nbp + c] = val;
      }
    }
    if (mode == 0) continue;
    __syncthreads();
    // ---- phase 2: fused partial product over the ROWS rows of this tile
    if (mode == 1) {
      // A^T Bout over the tile's rows: lane loads 4 consecutive columns of a row of its wave's
      // panel (32 bytes); value t feeds MFMA t (output row i stands for column 64 p + 4 i + t)
      for (int s = 0; s < ROWS / 4; s++) {
        const int rl = 4 * s + lk;
        const int64_t r = rbase + rl;
        double bop[MAXC];
#pragma unroll
        for (int q = 0; q < MAXC; q++) bop[q] = (q < ct) ? Wt[rl * nbp + q * 16 + li] : 0.0;
#pragma unroll
        for (int pi = 0; pi < MAXI; pi++) {
          const int pnl = wave + pi * WAVES;
          const int c0 = 64 * pnl + 4 * li;
          if (pnl < npan) {
            double a4[4];
            if (r < D && c0 < m) ld4(A + r * lda + c0, m - c0, a4);
            else a4[0] = a4[1] = a4[2] = a4[3] = 0.0;
#pragma unroll
            for (int t = 0; t < 4; t++)
#pragma unroll
              for (int q = 0; q < MAXC; q++)
                if (q < ct) pacc[pi][t][q] = mfma(a4[t], bop[q], pacc[pi][t][q]);
          }
        }
      }
    } else {
      // Gram of the tile: wave w takes row quads w, w+WAVES, ...; tiles (qi, qj) in pacc[qi][qj]
      for (int s = wave; s < ROWS / 4; s += WAVES) {
        const int rl = 4 * s + lk;
#pragma unroll
        for (int qi = 0; qi < MAXC; qi++) {
          if (qi >= ct) continue;
          const double aop = Wt[rl * nbp + qi * 16 + li];
#pragma unroll
          for (int qj = 0; qj < MAXC; qj++)
            if (qj < ct) pacc[0][qi][qj] = mfma(aop, Wt[rl * nbp + qj * 16 + li], pacc[0][qi][qj]);
        }
      }
    }
    __syncthreads();
  }
  if (mode == 0) return;
  double* out = part + (int64_t)blockIdx.x * (mode == 1 ? (int64_t)m * nb : (int64_t)nb * nb);
  if (mode == 1) {
#pragma unroll
    for (int pi = 0; pi < MAXI; pi++) {
      const int pnl = wave + pi * WAVES;
      if (pnl >= npan) continue;
#pragma unroll
      for (int t = 0; t < 4; t++)
#pragma unroll
        for (int q = 0; q < MAXC; q++) {
          if (q >= ct) continue;
#pragma unroll
          for (int v = 0; v < 4; v++) {
            const int i = 64 * pnl + 4 * (lk + 4 * v) + t, c = q * 16 + li;
            if (i < m && c < nb) out[i * nb + c] = pacc[pi][t][q][v];
          }
        }
    }
  } else {
    // reduce the per-wave Gram tiles through LDS, one wave after the other
    double* red = lds;  // nbp x nbp; all phases are done
    __syncthreads();
    for (int e = threadIdx.x; e < nbp * nbp; e += blockDim.x) red[e] = 0.0;
    for (int w = 0; w < WAVES; w++) {
      __syncthreads();
      if (wave != w) continue;
#pragma unroll
      for (int qi = 0; qi < MAXC; qi++) {
        if (qi >= ct) continue;
#pragma unroll
        for (int qj = 0; qj < MAXC; qj++) {
          if (qj >= ct) continue;
#pragma unroll
          for (int v = 0; v < 4; v++) red[(qi * 16 + lk + 4 * v) * nbp + qj * 16 + li] += pacc[0][qi][qj][v];
        }
      }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) {
      const int i = e / nb, c = e % nb;
      const double s = red[i * nbp + c];
      out[e] = s;
    }
  }
}

// ------------------------------------------------------------------ first CGS pass, fused
// Bout = Bin - A C together with part[g] = A^T Bout over the workgroup's rows, reading A once
// (nb <= 16, m <= 512). A tile of 16 rows is split by columns over 16 waves (at most 2 chunks
// of 16 columns each); each wave keeps its slice of C in registers, sums its share of A C into
// LDS, and parks its slice of the tile in LDS (rows padded by 4 values against bank conflicts)
// to read it back transposed for the projection, 2 consecutive columns per lane. The loads of
// A and Bin run PFD tiles ahead of the arithmetic, in PFD register buffers. Only the
// cross-wave sum needs the workgroup barriers.
template <class TA, class TI, int PFD>
__global__ __launch_bounds__(1024) void cgs_fused_kernel(const TA* __restrict__ A, int64_t lda, int m,
                                                         const double* __restrict__ C, const TI* Bin, int64_t ldi,
                                                         double* Bout, int64_t ldo, int nb, int64_t D,
                                                         double* __restrict__ part) {
  constexpr int WAVES = 16, KC = 2;
  extern __shared__ double lds[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int mt = (m + 15) >> 4;
  const int mp = mt * 16, asp = mp + 4;
  const int cpw = (mt + WAVES - 1) / WAVES;  // 16-column chunks per wave, <= KC
  const int kw0 = min(mp, wave * cpw * 16), kw1 = min(mp, kw0 + cpw * 16);
  const int nch = (kw1 - kw0) >> 4;
  const int erow = threadIdx.x >> 4, ec = threadIdx.x & 15;  // threads < 256: one element of the tile
  double* As = lds;                    // 16 x asp: the tile of A
  double* red = As + 16 * asp;         // WAVES x 16 x 16: partial products of the waves
  double* Wt = red + WAVES * 16 * 16;  // 16 x 16: the updated rows
  double cr[KC][4];
#pragma unroll
  for (int j = 0; j < KC; j++)
#pragma unroll
    for (int t = 0; t < 4; t++) {
      const int k = kw0 + 16 * j + 4 * lk + t;
      cr[j][t] = (j < nch && k < m && li < nb) ? C[k * nb + li] : 0.0;
    }
  d4 pacc[2] = {d4{0, 0, 0, 0}, d4{0, 0, 0, 0}};
  const int64_t ntiles = (D + 15) / 16;
  auto load = [&](int64_t tile, TA (&a)[KC][4], TI& bn) {
    if (tile >= ntiles) return;
    const int64_t ra = tile * 16 + li;
#pragma unroll
    for (int j = 0; j < KC; j++) {
      const int kk = kw0 + 16 * j + 4 * lk;
      if (j < nch && ra < D && kk < m) ld4raw(A + ra * lda + kk, m - kk, a[j]);
      else a[j][0] = a[j][1] = a[j][2] = a[j][3] = TA(0);
    }
    const int64_t r = tile * 16 + erow;
    bn = (threadIdx.x < 256 && r < D && ec < nb) ? Bin[r * ldi + ec] : TI(0);
  };
  // one tile from its buffer; the buffer is then refilled PFD tiles ahead
  auto body = [&](int64_t tile, TA (&a)[KC][4], TI& bn) {
    d4 acc = d4{0, 0, 0, 0};
#pragma unroll
    for (int j = 0; j < KC; j++) {
      if (j >= nch) continue;
      const int kk = kw0 + 16 * j + 4 * lk;
#pragma unroll
      for (int t = 0; t < 4; t++) {
        const double x = (double)a[j][t];
        As[li * asp + kk + t] = x;
        acc = mfma(x, cr[j][t], acc);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; v++) red[(wave * 16 + lk + 4 * v) * 16 + li] = acc[v];
    const double bcur = (double)bn;
    load(tile + (int64_t)PFD * gridDim.x, a, bn);
    __syncthreads();
    if (threadIdx.x < 256) {
      const int64_t r = tile * 16 + erow;
      double sum = 0.0;
#pragma unroll
      for (int w = 0; w < WAVES; w++) sum += red[(w * 16 + erow) * 16 + ec];
      double val = 0.0;
      if (r < D && ec < nb) {
        val = bcur - sum;
        Bout[r * ldo + ec] = val;
      }
      Wt[threadIdx.x] = val;
    }
    __syncthreads();
    // Wt and red are rewritten only after the next tile's first barrier, which every wave reaches
    // after this projection; each wave reads back only the slice of As it wrote itself.
    if (nch > 0) {
      const int c0 = kw0 + 2 * li;
#pragma unroll
      for (int sq = 0; sq < 4; sq++) {
        const int row = 4 * sq + lk;
        double a2[2];
#pragma unroll
        for (int t = 0; t < 2; t++) a2[t] = c0 < kw1 ? As[row * asp + c0 + t] : 0.0;
        const double bop = Wt[row * 16 + li];
#pragma unroll
        for (int t = 0; t < 2; t++) pacc[t] = mfma(a2[t], bop, pacc[t]);
      }
    }
  };
  TA a0[KC][4], a1[KC][4];
  TI b0 = TI(0), b1 = TI(0);
  load(blockIdx.x, a0, b0);
  if (PFD == 2) load(blockIdx.x + gridDim.x, a1, b1);
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += (int64_t)PFD * gridDim.x) {
    body(tile, a0, b0);
    if (PFD == 2 && tile + gridDim.x < ntiles) body(tile + gridDim.x, a1, b1);
  }
  double* out = part + (int64_t)blockIdx.x * m * nb;
#pragma unroll
  for (int t = 0; t < 2; t++)
#pragma unroll
    for (int v = 0; v < 4; v++) {
      const int col = kw0 + 2 * (lk + 4 * v) + t;
      if (col < m && col < kw1 && li < nb) out[(int64_t)col * nb + li] = pacc[t][v];
    }
}

// ------------------------------------------------------------------ Bout = Bin R  (R: nb x nb), optional Gram partial
template <class TI, class TO>
__global__ __launch_bounds__(256) void apply_small_kernel(const TI* Bin, int64_t ldi, const double* __restrict__ R,
                                                          TO* Bout, int64_t ldo, int nb, int64_t D, int gram,
                                                          double* __restrict__ part) {
  // tiles of `rows` rows (rows * nb = 2048 values); thread t owns column t % nb of rows t / nb,
  // t / nb + 256 / nb, ...; the Gram partial of the tile is formed from the outputs in LDS,
  // one (i, j) pair per thread.
  extern __shared__ double lds[];
  double* Rs = lds;                 // nb x nb
  const int rows = 2048 / nb;
  double* tile = lds + nb * nb;     // rows x nb inputs
  double* outt = tile + rows * nb;  // rows x nb outputs
  for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) Rs[e] = R[e];
  const int npair = nb * nb;
  double g[16];
  for (int q = 0; q < 16; q++) g[q] = 0.0;
  __syncthreads();
  const int64_t ntiles = (D + rows - 1) / rows;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t r0 = t * rows;
    for (int e = threadIdx.x; e < rows * nb; e += blockDim.x) {
      const int64_t r = r0 + e / nb;
      tile[e] = (r < D) ? ld(Bin + r * ldi + e % nb) : 0.0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < rows * nb; e += blockDim.x) {
      const int rl = e / nb, c = e % nb;
      const double* tr = tile + rl * nb;
      double s = 0.0;
      for (int k = 0; k < nb; k++) s += tr[k] * Rs[k * nb + c];
      const TO so = (TO)s;  // the Gram partial is that of the stored (possibly rounded) values
      outt[e] = (double)so;
      const int64_t r = r0 + rl;
      if (r < D) Bout[r * ldo + c] = so;
    }
    if (gram) {
      __syncthreads();
      for (int q = 0; q < 16; q++) {
        const int pidx = threadIdx.x + q * blockDim.x;
        if (pidx < npair) {
          const int i = pidx / nb, j = pidx % nb;
          double s = 0.0;
          for (int rl = 0; rl < rows; rl++) s += outt[rl * nb + i] * outt[rl * nb + j];
          g[q] += s;
        }
      }
    }
    __syncthreads();
  }
  if (gram) {
    double* out = part + (int64_t)blockIdx.x * npair;
    for (int q = 0; q < 16; q++) {
      const int pidx = threadIdx.x + q * blockDim.x;
      if (pidx < npair) out[pidx] = g[q];
    }
  }
}

// ------------------------------------------------------------------ Cholesky of the nb x nb Gram matrix
// Sums G partials, factors G = R^T R (R upper, positive diagonal), inverts R,
// and optionally forms beta = R * Rprev. status[0] = 0 ok, 1 not positive definite.
__global__ __launch_bounds__(256) void chol_kernel(const double* __restrict__ part, int G, int nb, double* R,
                                                   double* Rinv, const double* Rprev, double* beta, int* status) {
  extern __shared__ double lds[];
  double* A = lds;            // nb x nb
  double* Ri = lds + nb * nb; // nb x nb
  const int n2 = nb * nb;
  for (int e = threadIdx.x; e < n2; e += blockDim.x) {
    double s = 0.0;
    for (int g = 0; g < G; g++) s += part[(int64_t)g * n2 + e];
    A[e] = s;
  }
  __syncthreads();
  __shared__ int bad;
  __shared__ double dmax;
  if (threadIdx.x == 0) {
    bad = 0;
    double mx = 0.0;
    for (int i = 0; i < nb; i++) mx = fmax(mx, fabs(A[i * nb + i]));
    dmax = mx;
  }
  __syncthreads();
  // right-looking Cholesky on the upper triangle
  for (int k = 0; k < nb; k++) {
    if (threadIdx.x == 0) {
      const double piv = A[k * nb + k];
      // beyond a condition number of ~1e7 Cholesky QR loses accuracy: take the column-wise path
      if (!(piv > 1e-14 * dmax) || !(dmax > 0.0)) bad = 1;
      A[k * nb + k] = sqrt(fmax(piv, 1e-300));
    }
    __syncthreads();
    const double rkk = A[k * nb + k];
    for (int j = k + 1 + threadIdx.x; j < nb; j += blockDim.x) A[k * nb + j] /= rkk;
    __syncthreads();
    for (int e = threadIdx.x; e < n2; e += blockDim.x) {
      const int i = e / nb, j = e % nb;
      if (i > k && j >= i) A[i * nb + j] -= A[k * nb + i] * A[k * nb + j];
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < n2; e += blockDim.x) {
    const int i = e / nb, j = e % nb;
    if (j < i) A[e] = 0.0;
  }
  __syncthreads();
  // inverse of the upper-triangular R, column by column (one thread per column)
  for (int j = threadIdx.x; j < nb; j += blockDim.x) {
    for (int i = 0; i < nb; i++) Ri[i * nb + j] = 0.0;
    Ri[j * nb + j] = 1.0 / A[j * nb + j];
    for (int i = j - 1; i >= 0; i--) {
      double s = 0.0;
      for (int k = i + 1; k <= j; k++) s += A[i * nb + k] * Ri[k * nb + j];
      Ri[i * nb + j] = -s / A[i * nb + i];
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < n2; e += blockDim.x) {
    R[e] = A[e];
    Rinv[e] = Ri[e];
    if (beta) {
      const int i = e / nb, j = e % nb;
      double s = 0.0;
      for (int k = 0; k < nb; k++) s += A[i * nb + k] * Rprev[k * nb + j];
      beta[e] = s;
    }
  }
  if (threadIdx.x == 0) status[0] = bad;
}

// ------------------------------------------------------------------ Y = A U (row-wise), optionally in place
// Y[r, 0:ncol] = A[r, 0:m] U[0:m, 0:ncol] (U row-major, ld ldu). In place (Y == A) is allowed:
// every workgroup reads all of its rows before it writes them. If vsrc >= 0, columns
// [vsrc, vsrc+nv) of A are copied to columns [vdst, vdst+nv) of Y after the product.
template <class TA, class TY, int NT>
__global__ __launch_bounds__(512) void rowgemm_kernel(const TA* A, int64_t lda, int m, const double* __restrict__ U,
                                                      int64_t ldu, int ncol, TY* Y, int64_t ldy, int64_t D, int vsrc,
                                                      int vdst, int nv) {
  // U is staged by chunks of KC rows into two alternating LDS buffers and A is loaded one
  // chunk ahead in registers, so each chunk costs one barrier and its loads overlap the
  // previous chunk's MFMAs
  constexpr int WAVES = 8, ROWS = WAVES * 16, KC = 16, UW = NT * 16;
  constexpr int UPT = (KC * UW + WAVES * 64 - 1) / (WAVES * 64);  // U values per thread and chunk
  extern __shared__ double lds[];
  double* Us = lds;                 // 2 x KC x UW
  double* Vs = lds + 2 * KC * UW;   // ROWS x nv (copy of the moved block)
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int ctile = (ncol + 15) >> 4;
  const int nk = (m + KC - 1) / KC;
  const int64_t ntiles = (D + ROWS - 1) / ROWS;
  auto load_u = [&](int k0, double (&u)[UPT]) {
#pragma unroll
    for (int i = 0; i < UPT; i++) {
      const int e = threadIdx.x + i * WAVES * 64;
      const int k = k0 + e / UW, c = e % UW;
      u[i] = (e < KC * UW && k < m && c < ncol) ? U[k * ldu + c] : 0.0;
    }
  };
  auto store_u = [&](int buf, const double (&u)[UPT]) {
#pragma unroll
    for (int i = 0; i < UPT; i++) {
      const int e = threadIdx.x + i * WAVES * 64;
      if (e < KC * UW) Us[buf * KC * UW + e] = u[i];
    }
  };
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t rbase = tile * ROWS;
    if (vsrc >= 0) {
      for (int e = threadIdx.x; e < ROWS * nv; e += blockDim.x) {
        const int64_t r = rbase + e / nv;
        Vs[e] = (r < D) ? ld(A + r * lda + vsrc + e % nv) : 0.0;
      }
    }
    d4 acc[NT];
#pragma unroll
    for (int q = 0; q < NT; q++) acc[q] = d4{0, 0, 0, 0};
    const int64_t ra = rbase + wave * 16 + li;
    const int kk = 4 * lk;
    auto load_a = [&](int k0, double (&a4)[4]) {
      if (ra < D && k0 + kk < m) ld4(A + ra * lda + k0 + kk, m - (k0 + kk), a4);
      else a4[0] = a4[1] = a4[2] = a4[3] = 0.0;
    };
    double u[UPT], a4[4], an[4];
    load_u(0, u);
    store_u(0, u);
    load_a(0, a4);
    __syncthreads();
    for (int s = 0; s < nk; s++) {
      const int k0 = s * KC, buf = s & 1;
      const bool more = s + 1 < nk;
      if (more) {
        load_u(k0 + KC, u);
        load_a(k0 + KC, an);
      }
      const double* ub = Us + buf * KC * UW;
#pragma unroll
      for (int t = 0; t < 4; t++) {
#pragma unroll
        for (int q = 0; q < NT; q++)
          if (q < ctile) acc[q] = mfma(a4[t], ub[(kk + t) * UW + q * 16 + li], acc[q]);
      }
      if (more) store_u(buf ^ 1, u);
      __syncthreads();  // the last one also orders every read of the tile's A before the writes of Y
#pragma unroll
      for (int t = 0; t < 4; t++) a4[t] = an[t];
    }
#pragma unroll
    for (int q = 0; q < NT; q++) {
      if (q >= ctile) continue;
#pragma unroll
      for (int v = 0; v < 4; v++) {
        const int64_t r = rbase + wave * 16 + lk + 4 * v;
        const int c = q * 16 + li;
        if (r < D && c < ncol) Y[r * ldy + c] = (TY)acc[q][v];
      }
    }
    if (vsrc >= 0) {
      for (int e = threadIdx.x; e < ROWS * nv; e += blockDim.x) {
        const int64_t r = rbase + e / nv;
        if (r < D) Y[r * ldy + vdst + e % nv] = (TY)Vs[e];
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ small helpers
// Standard normals: element (i, c) is normal number i*nb + c of splitmix64(seed) + Box-Muller.
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t counter) {
  uint64_t z = seed + (counter + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

template <class T>
__global__ void random_kernel(T* out, int64_t ld, int64_t D, int nb, uint64_t seed) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < D * nb; e += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t k = (uint64_t)e;
    const double u1 = ((double)(splitmix64(seed, 2 * k) >> 11) + 1.0) * (1.0 / 9007199254740992.0);
    const double u2 = ((double)(splitmix64(seed, 2 * k + 1) >> 11) + 1.0) * (1.0 / 9007199254740992.0);
    const double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
    out[(e / nb) * ld + e % nb] = (T)z;
  }
}

template <class T>
__global__ void mask_rows_kernel(T* X, int64_t ld, int64_t D, int ncol, const double* __restrict__ mask) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < D * ncol; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / ncol;
    if (mask[r] == 0.0) X[r * ld + (e - r * ncol)] = T(0);
  }
}

template <class TS, class TD>
__global__ void copy_cols_kernel(const TS* src, int64_t lds_, TD* dst, int64_t ldd, int64_t D, int ncol) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < D * ncol; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / ncol;
    const int c = (int)(e % ncol);
    dst[r * ldd + c] = (TD)src[r * lds_ + c];
  }
}

// T-matrix bookkeeping of Alg. 4 (device-resident T, leading dimension ldt)
__global__ void t_alpha_kernel(double* T, int ldt, int c0, int nb, const double* C1) {
  // alpha_k = V_k^T W is rows c0..c0+nb of C1 (m x nb); symmetrised
  const int e = threadIdx.x + blockIdx.x * blockDim.x;
  if (e >= nb * nb) return;
  const int i = e / nb, j = e % nb;
  T[(c0 + i) * ldt + c0 + j] = 0.5 * (C1[(c0 + i) * nb + j] + C1[(c0 + j) * nb + i]);
}

__global__ void t_column_kernel(const double* T, int ldt, int c0, int r_lo, int nb, double* C) {
  // rows r_lo..c0-1 of column block c0 of T (the couplings of V_k to the earlier vectors)
  const int e = threadIdx.x + blockIdx.x * blockDim.x;
  if (e >= (c0 - r_lo) * nb) return;
  const int r = r_lo + e / nb, c = e % nb;
  C[r * nb + c] = T[r * ldt + c0 + c];
}

__global__ void t_beta_kernel(double* T, int ldt, int c0, int m, int nb, const double* beta) {
  const int e = threadIdx.x + blockIdx.x * blockDim.x;
  if (e >= nb * nb) return;
  const int i = e / nb, j = e % nb;
  T[(m + i) * ldt + c0 + j] = beta[i * nb + j];
  T[(c0 + j) * ldt + m + i] = beta[i * nb + j];
}

// residual norms rho_i = || beta U[m-nb:m, i] || for i < n
__global__ void resid_kernel(const double* beta, int nb, const double* U, int ldu, int m, int n, double* rho) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int a = 0; a < nb; a++) {
    double x = 0.0;
    for (int b = 0; b < nb; b++) x += beta[a * nb + b] * U[(m - nb + b) * ldu + i];
    s += x * x;
  }
  rho[i] = sqrt(s);
}

// restart: T := [diag(theta_1..ls)  r^T ; r  .], r = beta U[m-nb:m, 0:ls] (T zeroed first)
__global__ void t_restart_fill_kernel(double* T, int ldt, const double* theta, int ls, const double* beta, int nb,
                                      const double* U, int ldu, int m) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < ls) T[e * ldt + e] = theta[e];
  if (e < nb * ls) {
    const int a = e / ls, k = e % ls;
    double s = 0.0;
    for (int b = 0; b < nb; b++) s += beta[a * nb + b] * U[(m - nb + b) * ldu + k];
    T[(ls + a) * ldt + k] = s;
    T[k * ldt + ls + a] = s;
  }
}

// ------------------------------------------------------------------ host launchers
static int grid_for(int64_t rows, int64_t rows_per_wg, int cap) {
  int64_t g = (rows + rows_per_wg - 1) / rows_per_wg;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

template <class TA, class TB>
void tn(const TA* A, int64_t lda, int m, const TB* B, int64_t ldb, int nb, int64_t D, double* C, Scratch& s,
        hipStream_t st) {
  TRBL_REQUIRE(m >= 1 && nb >= 1 && nb <= 64, TRBL_E_INVALID, "projection shape out of range");
  const int ct = (nb + 15) / 16;
  const int np = ct == 1 ? std::min(2, (m + 63) / 64) : 1;  // panels of 64 columns per workgroup
  const int ny = (m + 64 * np - 1) / (64 * np);
  int G = grid_for(D, 512, std::max(64, 1024 / ny));
  int64_t rows_per = ((D + G - 1) / G + 15) / 16 * 16;
  G = (int)((D + rows_per - 1) / rows_per);
  double* part = s.partials((size_t)G * m * nb);
  const dim3 grid(G, ny);
#define TN_LAUNCH(NP, MC) \
  hipLaunchKernelGGL((tn_partial_kernel<TA, TB, NP, MC>), grid, dim3(256), 0, st, A, lda, m, B, ldb, nb, D, rows_per, part)
  if (ct == 1) {
    if (np == 1) TN_LAUNCH(1, 1);
    else TN_LAUNCH(2, 1);
  } else if (ct == 2) {
    TN_LAUNCH(1, 2);
  } else {
    TN_LAUNCH(1, 4);
  }
#undef TN_LAUNCH
  const int64_t len = (int64_t)m * nb;
  hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)((len + 15) / 16)), dim3(256), 0, st, part, G, len, C);
  TRBL_HIP(hipGetLastError());
}

template <class TA, class TI, class TO>
void update(const TA* A, int64_t lda, int m, const double* C, const TI* Bin, int64_t ldi, TO* Bout, int64_t ldo,
            int nb, int64_t D, int mode, double* Pout, Scratch& s, hipStream_t st, TO* Bout2, int64_t ldo2) {
  TRBL_REQUIRE(m >= 1 && m <= 768 && nb >= 1 && nb <= 64, TRBL_E_INVALID, "projection shape out of range");
  TRBL_REQUIRE(!Bout2 || (mode != 1 && Bout2 != Bout), TRBL_E_INVALID, "second output only for modes 0 and 2");
  const int mt = (m + 15) / 16, ct = (nb + 15) / 16, npan = (m + 63) / 64;
  if constexpr (sizeof(TO) == 8) {
  if (mode == 1 && mt <= 32 && ct == 1 && Bin) {  // one pass over A for the update and the projection
    const size_t shmf = (size_t)(16 * (mt * 16 + 4) + 16 * 16 * 16 + 16 * 16) * sizeof(double);
    const int G = grid_for(D, 16, 256);  // one resident workgroup of 16 waves per CU
    double* part = s.partials((size_t)G * m * nb);
    constexpr int PFD = sizeof(TA) == 4 ? 2 : 1;  // FP32 panels: half the bytes per tile, twice the tiles in flight
    hipLaunchKernelGGL((cgs_fused_kernel<TA, TI, PFD>), dim3(G), dim3(1024), shmf, st, A, lda, m, C, Bin, ldi, Bout,
                       ldo, nb, D, part);
    const int64_t plen = (int64_t)m * nb;
    if (Pout)
      hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)((plen + 15) / 16)), dim3(256), 0, st, part, G, plen,
                         Pout);
    s.last_G = G;
    s.last_part = part;
    TRBL_HIP(hipGetLastError());
    return;
  }
  }
  auto shm_for = [&](int waves) {
    size_t b = (size_t)(mt * 16 * ct * 16 + waves * 16 * ct * 16) * sizeof(double);
    return std::max(b, (size_t)ct * 16 * ct * 16 * sizeof(double));
  };
  if (shm_for(4) > 160 * 1024) {
    // C (m x nb) does not fit the LDS next to the tile: the columns of A in chunks, the first
    // from Bin, the rest in place on Bout; the fused products after the last chunk (Gram) or
    // separately (A^T Bout)
    const int mmax = (int)((160 * 1024 / sizeof(double) - 4 * 16 * ct * 16) / (ct * 16)) / 16 * 16;
    TRBL_REQUIRE(mmax >= 16 && Bin != nullptr && !Bout2, TRBL_E_INVALID, "update tile does not fit in LDS");
    for (int k0 = 0; k0 < m; k0 += mmax) {
      const int mc = std::min(mmax, m - k0);
      const bool last = k0 + mc >= m;
      if (k0 == 0)
        update<TA, TI, TO>(A + k0, lda, mc, C + (size_t)k0 * nb, Bin, ldi, Bout, ldo, nb, D,
                           last && mode == 2 ? 2 : 0, nullptr, s, st);
      else
        update<TA, TO, TO>(A + k0, lda, mc, C + (size_t)k0 * nb, Bout, ldo, Bout, ldo, nb, D,
                           last && mode == 2 ? 2 : 0, nullptr, s, st);
    }
    if (mode == 1) {
      TRBL_REQUIRE(Pout != nullptr, TRBL_E_INVALID, "projection output missing");
      tn<TA, TO>(A, lda, m, Bout, ldo, nb, D, Pout, s, st);
    }
    return;
  }
  const int waves = (shm_for(8) <= 160 * 1024) ? 8 : 4;
  const size_t shm = shm_for(waves);
  int G = grid_for(D, waves * 16 * 4, 1024);
  const int64_t plen = mode == 1 ? (int64_t)m * nb : (int64_t)nb * nb;
  double* part = mode ? s.partials((size_t)G * plen) : nullptr;
  const int mi = (npan + waves - 1) / waves;  // 64-column panels per wave (mode 1)
#define UPD_LAUNCH(W, MI, MC)                                                                                     \
  hipLaunchKernelGGL((update_kernel<TA, TI, TO, W, MI, MC>), dim3(G), dim3(W * 64), shm, st, A, lda, m, C, Bin, ldi, \
                     Bout, ldo, nb, D, mode, part, Bout2, ldo2)
  if (waves == 8) {
    if (ct == 1) {
      if (mi <= 1) UPD_LAUNCH(8, 1, 1);
      else UPD_LAUNCH(8, 2, 1);
    } else if (ct == 2) {
      if (mi <= 1) UPD_LAUNCH(8, 1, 2);
      else UPD_LAUNCH(8, 2, 2);
    } else {
      if (mi <= 1) UPD_LAUNCH(8, 1, 4);
      else UPD_LAUNCH(8, 2, 4);
    }
  } else {
    if (ct <= 2) UPD_LAUNCH(4, 3, 2);
    else UPD_LAUNCH(4, 3, 4);
  }
#undef UPD_LAUNCH
  if (mode) {
    if (Pout)
      hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)((plen + 15) / 16)), dim3(256), 0, st, part, G,
                         plen, Pout);
    s.last_G = G;
    s.last_part = part;
  }
  TRBL_HIP(hipGetLastError());
}

template <class TI, class TO>
void apply_small(const TI* Bin, int64_t ldi, const double* R, TO* Bout, int64_t ldo, int nb, int64_t D, bool gram,
                 Scratch& s, hipStream_t st, TO* Bout2, int64_t ldo2) {
  if constexpr (sizeof(TO) == 8 || sizeof(TI) == sizeof(TO)) {
    // FP64 output, or FP32 in and out: the MFMA row-streaming kernel, Bout = Bin R (+ Gram)
    update<TI, TI, TO>(Bin, ldi, nb, R, nullptr, 0, Bout, ldo, nb, D, gram ? 2 : 0, nullptr, s, st, Bout2, ldo2);
    return;
  }
  TRBL_REQUIRE(!Bout2, TRBL_E_INVALID, "second output only for FP64 or same-precision products");
  const int rows = 2048 / nb;
  const int G = grid_for(D, rows * 4, 1024);
  double* part = gram ? s.partials((size_t)G * nb * nb) : nullptr;
  const size_t shm = (size_t)(nb * nb + 2 * rows * nb) * sizeof(double);
  hipLaunchKernelGGL((apply_small_kernel<TI, TO>), dim3(G), dim3(256), shm, st, Bin, ldi, R, Bout, ldo, nb, D,
                     gram ? 1 : 0, part);
  if (gram) {
    s.last_G = G;
    s.last_part = part;
  }
  TRBL_HIP(hipGetLastError());
}

void chol(const double* part, int G, int nb, double* R, double* Rinv, const double* Rprev, double* beta, int* status,
          hipStream_t st) {
  const size_t shm = 2 * (size_t)nb * nb * sizeof(double);
  if (G > 1) {  // sum the partials into slice 0 (each block reads its own columns before writing them)
    const int64_t len = (int64_t)nb * nb;
    hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)((len + 15) / 16)), dim3(256), 0, st, part, G, len,
                       const_cast<double*>(part));
    G = 1;
  }
  hipLaunchKernelGGL(chol_kernel, dim3(1), dim3(256), shm, st, part, G, nb, R, Rinv, Rprev, beta, status);
  TRBL_HIP(hipGetLastError());
}

template <class TA, class TY>
void rowgemm(const TA* A, int64_t lda, int m, const double* U, int64_t ldu, int ncol, TY* Y, int64_t ldy, int64_t D,
             int vsrc, int vdst, int nv, hipStream_t st, TY* tmp, int64_t tmp_elems) {
  const int G = grid_for(D, 128, 2048);
  const int nt = (ncol + 15) / 16;
  auto shm = [&](int NT) { return (size_t)(2 * 16 * NT * 16 + 128 * std::max(nv, 1)) * sizeof(double); };
  if (nt <= 4)
    hipLaunchKernelGGL((rowgemm_kernel<TA, TY, 4>), dim3(G), dim3(512), shm(4), st, A, lda, m, U, ldu, ncol, Y, ldy,
                       D, vsrc, vdst, nv);
  else if (nt <= 8)
    hipLaunchKernelGGL((rowgemm_kernel<TA, TY, 8>), dim3(G), dim3(512), shm(8), st, A, lda, m, U, ldu, ncol, Y, ldy,
                       D, vsrc, vdst, nv);
  else if (nt <= 13)
    hipLaunchKernelGGL((rowgemm_kernel<TA, TY, 13>), dim3(G), dim3(512), shm(13), st, A, lda, m, U, ldu, ncol, Y,
                       ldy, D, vsrc, vdst, nv);
  else {
    // wide outputs: column groups of 13 tiles. In place, a group would overwrite columns that the
    // next group still reads, so rows go through tmp in chunks: each chunk is computed out of
    // place, then copied back with its part of the moved block before the next chunk is read.
    auto groups = [&](const TA* a, TY* y, int64_t ly, int64_t rows) {
      const int g = grid_for(rows, 128, 2048);
      for (int c0 = 0; c0 < ncol; c0 += 13 * 16) {
        const int nc = std::min(13 * 16, ncol - c0);
        hipLaunchKernelGGL((rowgemm_kernel<TA, TY, 13>), dim3(g), dim3(512), shm(13), st, a, lda, m, U + c0, ldu, nc,
                           y + c0, ly, rows, -1, 0, 0);
      }
    };
    if ((const void*)A != (const void*)Y) {
      groups(A, Y, ldy, D);
      if (vsrc >= 0) copy_cols<TA, TY>(A + vsrc, lda, Y + vdst, ldy, D, nv, st);
    } else {
      // the moved block of a chunk is parked in tmp too (its source and destination may overlap)
      const int nvv = vsrc >= 0 ? nv : 0;
      TRBL_REQUIRE(tmp && tmp_elems >= (int64_t)(ncol + nvv), TRBL_E_INVALID,
                   "in-place product wider than 208 columns needs a work buffer");
      TRBL_REQUIRE(vsrc < 0 || vdst >= ncol, TRBL_E_INVALID, "moved block inside the product's columns");
      int64_t chunk = tmp_elems / (ncol + nvv);
      if (chunk >= 128) chunk = chunk / 128 * 128;  // whole row tiles of the kernel
      chunk = std::min<int64_t>(D, chunk);
      TY* tv = tmp + chunk * ncol;
      for (int64_t r0 = 0; r0 < D; r0 += chunk) {
        const int64_t rows = std::min(chunk, D - r0);
        groups(A + r0 * lda, tmp, ncol, rows);
        if (nvv) copy_cols<TA, TY>(A + r0 * lda + vsrc, lda, tv, nv, rows, nv, st);
        copy_cols<TY, TY>(tmp, ncol, Y + r0 * ldy, ldy, rows, ncol, st);
        if (nvv) copy_cols<TY, TY>(tv, nv, Y + r0 * ldy + vdst, ldy, rows, nv, st);
      }
    }
  }
  TRBL_HIP(hipGetLastError());
}

template <class T>
void random_block(T* out, int64_t ld, int64_t D, int nb, uint64_t seed, hipStream_t st) {
  const int64_t n = D * nb;
  hipLaunchKernelGGL(random_kernel<T>, dim3(elementwise_grid(n)), dim3(256), 0, st, out, ld, D, nb, seed);
  TRBL_HIP(hipGetLastError());
}

template <class T>
void mask_rows(T* X, int64_t ld, int64_t D, int ncol, const double* mask, hipStream_t st) {
  if (!mask) return;
  const int64_t n = D * ncol;
  hipLaunchKernelGGL(mask_rows_kernel<T>, dim3(elementwise_grid(n)), dim3(256), 0, st, X, ld, D, ncol, mask);
  TRBL_HIP(hipGetLastError());
}

template <class TS, class TD>
void copy_cols(const TS* src, int64_t lds_, TD* dst, int64_t ldd, int64_t D, int ncol, hipStream_t st) {
  const int64_t n = D * ncol;
  hipLaunchKernelGGL((copy_cols_kernel<TS, TD>), dim3(elementwise_grid(n)), dim3(256), 0, st, src, lds_, dst, ldd, D,
                     ncol);
  TRBL_HIP(hipGetLastError());
}

void t_alpha(double* T, int ldt, int c0, int nb, const double* C1, hipStream_t st) {
  hipLaunchKernelGGL(t_alpha_kernel, dim3((nb * nb + 255) / 256), dim3(256), 0, st, T, ldt, c0, nb, C1);
}
void t_column(const double* T, int ldt, int c0, int r_lo, int nb, double* C, hipStream_t st) {
  if (c0 <= r_lo) return;
  hipLaunchKernelGGL(t_column_kernel, dim3(((c0 - r_lo) * nb + 255) / 256), dim3(256), 0, st, T, ldt, c0, r_lo, nb, C);
  TRBL_HIP(hipGetLastError());
}
void t_beta(double* T, int ldt, int c0, int m, int nb, const double* beta, hipStream_t st) {
  hipLaunchKernelGGL(t_beta_kernel, dim3((nb * nb + 255) / 256), dim3(256), 0, st, T, ldt, c0, m, nb, beta);
}
void resid(const double* beta, int nb, const double* U, int ldu, int m, int n, double* rho, hipStream_t st) {
  hipLaunchKernelGGL(resid_kernel, dim3((n + 255) / 256), dim3(256), 0, st, beta, nb, U, ldu, m, n, rho);
}
void t_restart(double* T, int ldt, int lm, const double* theta, int ls, const double* beta, int nb, const double* U,
               int ldu, int m, hipStream_t st) {
  TRBL_HIP(hipMemsetAsync(T, 0, sizeof(double) * (size_t)lm * ldt, st));
  const int n = std::max(ls, nb * ls);
  hipLaunchKernelGGL(t_restart_fill_kernel, dim3((n + 255) / 256), dim3(256), 0, st, T, ldt, theta, ls, beta, nb, U,
                     ldu, m);
  TRBL_HIP(hipGetLastError());
}

// explicit instantiations
template void tn<double, double>(const double*, int64_t, int, const double*, int64_t, int, int64_t, double*, Scratch&,
                                 hipStream_t);
template void tn<float, float>(const float*, int64_t, int, const float*, int64_t, int, int64_t, double*, Scratch&,
                               hipStream_t);
template void tn<float, double>(const float*, int64_t, int, const double*, int64_t, int, int64_t, double*, Scratch&,
                                hipStream_t);
template void tn<double, float>(const double*, int64_t, int, const float*, int64_t, int, int64_t, double*, Scratch&,
                                hipStream_t);
template void update<double, double, double>(const double*, int64_t, int, const double*, const double*, int64_t,
                                             double*, int64_t, int, int64_t, int, double*,
                                             Scratch&, hipStream_t, double*, int64_t);
template void update<float, float, double>(const float*, int64_t, int, const double*, const float*, int64_t, double*,
                                           int64_t, int, int64_t, int, double*,
                                           Scratch&, hipStream_t, double*, int64_t);
template void update<float, double, double>(const float*, int64_t, int, const double*, const double*, int64_t,
                                            double*, int64_t, int, int64_t, int, double*,
                                            Scratch&, hipStream_t, double*, int64_t);
template void update<float, float, float>(const float*, int64_t, int, const double*, const float*, int64_t, float*,
                                          int64_t, int, int64_t, int, double*, Scratch&, hipStream_t, float*, int64_t);
template void apply_small<double, double>(const double*, int64_t, const double*, double*, int64_t, int, int64_t, bool,
                                          Scratch&, hipStream_t, double*, int64_t);
template void apply_small<double, float>(const double*, int64_t, const double*, float*, int64_t, int, int64_t, bool,
                                         Scratch&, hipStream_t, float*, int64_t);
template void apply_small<float, float>(const float*, int64_t, const double*, float*, int64_t, int, int64_t, bool,
                                        Scratch&, hipStream_t, float*, int64_t);
template void apply_small<float, double>(const float*, int64_t, const double*, double*, int64_t, int, int64_t, bool,
                                         Scratch&, hipStream_t, double*, int64_t);
template void rowgemm<double, double>(const double*, int64_t, int, const double*, int64_t, int, double*, int64_t,
                                      int64_t, int, int, int, hipStream_t, double*, int64_t);
template void rowgemm<float, float>(const float*, int64_t, int, const double*, int64_t, int, float*, int64_t, int64_t,
                                    int, int, int, hipStream_t, float*, int64_t);
template void rowgemm<float, double>(const float*, int64_t, int, const double*, int64_t, int, double*, int64_t,
                                     int64_t, int, int, int, hipStream_t, double*, int64_t);
template void random_block<double>(double*, int64_t, int64_t, int, uint64_t, hipStream_t);
template void random_block<float>(float*, int64_t, int64_t, int, uint64_t, hipStream_t);
template void mask_rows<double>(double*, int64_t, int64_t, int, const double*, hipStream_t);
template void mask_rows<float>(float*, int64_t, int64_t, int, const double*, hipStream_t);
template void copy_cols<double, double>(const double*, int64_t, double*, int64_t, int64_t, int, hipStream_t);
template void copy_cols<float, float>(const float*, int64_t, float*, int64_t, int64_t, int, hipStream_t);
template void copy_cols<float, double>(const float*, int64_t, double*, int64_t, int64_t, int, hipStream_t);
template void copy_cols<double, float>(const double*, int64_t, float*, int64_t, int64_t, int, hipStream_t);

}  // namespace trbl
