// On-the-fly block H.V (App. B) and device-side basis indexing (App. A).
//
// W = H V for nb vectors stored row-major [D][ld]. Every output row
// (p', n') of a proton-major block b' is produced by one lane:
//   identical-particle part  sum_p  Hpp[p',p] V[p, n']   (same block)
//                          + sum_n  Hnn[n',n] V[p', n]   (same block)
//   proton-neutron part      sum over proton jumps p' -> p (remove a, add c)
//                            and neutron jumps n' -> n (remove b, add d) with
//                            opposite change of M and the same parity flip:
//                            s_p s_n h(a b c d) V[p, n]   (source block b)
// (the factorisation c+_a c+_b c_d c_c = (c+_a c_c)_p (c+_b c_d)_n of App. B,
// with Jordan-Wigner signs counted inside each species). Jumps include the
// number operators (a == c), so the pn diagonal needs no special case. The
// element h is generated from the class tables for every (p', n') and reused
// across the C vectors of a column tile held in the lane's registers.
//
// The rows kernel owns one target proton row p' (one workgroup, one lane per
// target neutron n'). The source rows V[p, :, tile] of its proton jumps are
// streamed through two LDS buffers: while the lanes gather from one buffer,
// the next source row is copied into the other by the global->LDS DMA of
// gfx950 (no registers involved). Rows are stored plainly; a lane reads the
// 16-byte chunks of a row starting at chunk (lane mod chunks-per-row), so the
// lanes of a wavefront that gather from random rows still hit different LDS
// banks at each step. Accumulator slot t of lane l therefore holds column chunk
// (t + l) mod chunks-per-row, which the final store undoes.
#pragma once
#include "internal.h"

namespace trbl {

template <class T>
struct HVArgs {
  const T* V;
  T* W;
  int64_t ldv, ldw;
  int nb, ncl, tjmax, nblocks;
  int nnum;              // neutron number operators merged in the diagonal class (0: none)
  int C, ntile, nchunk;  // column tile width, column tiles, target chunks per row/column
  int dma;               // source rows copied by global->LDS DMA (16-byte aligned rows)
  int64_t nn_total;
  const int* blk_dp;
  const int* blk_dn;
  const int64_t* blk_off;
  const int* blk_p0;
  const int* blk_n0;
  const int* src_blk;
  const int* pj_start;
  const int* pj_idx;
  const int* pj_meta;
  const int* pg_start;  // per proton SD: first jump group
  const int* pg_desc;   // jump groups, 4 ints each: class, first jump, end jump, source row
  const int* nj_start;  // class-major: [cls * (nn_total + 1) + g]
  const int2* nj_pack;  // (source local index, op << 1 | sign)
  const int* h_off;
  const int* h_ncol;
  const T* h;
  const int* pe_off;  // sliced-ELL identical-particle operators (proton, neutron)
  const int* pe_w;
  const int* pe_col;
  const T* pe_val;
  const int* ne_off;
  const int* ne_w;
  const int* ne_col;
  const T* ne_val;
  const int* blk_pslice0;
  const int* blk_nslice0;
  const int* bin_blocks;   // rows kernel: blocks of this launch
  const int64_t* bin_item0;  // rows kernel: first work item of each of them (bin_nblk + 1)
  int bin_nblk;
  const int64_t* citem0;  // per block: first work item (columns kernel)
};

// Work item -> (block, row, column tile, target chunk); consecutive items go to one XCD.
__device__ __forceinline__ int64_t xcd_item(int64_t bid, int64_t n) {
  const int64_t per = (n + 7) / 8;
  const int64_t x = bid % 8, q = bid / 8;
  return x * per + q;
}

__device__ __forceinline__ int find_block(const int64_t* item0, int nblocks, int64_t item) {
  int lo = 0, hi = nblocks - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (item0[mid] <= item) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// ---------------------------------------------------------------- columns kernel helpers
// padded LDS row stride (elements): > C and a multiple of 16 bytes so a row slice is 16-byte aligned
template <class T, int C>
constexpr int row_stride() {
  return sizeof(T) == 8 ? (C >= 2 ? C + 2 : 2) : (C >= 4 ? C + 4 : 4);
}

// lds[r * RS + c] = src[r * rstride + c] for r < nrows, c < C (zero beyond cvalid)
template <class T, int C>
__device__ __forceinline__ void stage(T* lds, const T* src, int64_t rstride, int nrows, int cvalid) {
  constexpr int RS = row_stride<T, C>();
  const int n = nrows * C;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    const int r = e / C, c = e % C;
    lds[r * RS + c] = (c < cvalid) ? src[(int64_t)r * rstride + c] : T(0);
  }
}

template <class T, int C>
__device__ __forceinline__ void axpy_row(T (&acc)[C], T coef, const T* x) {
#pragma unroll
  for (int c = 0; c < C; c++) acc[c] += coef * x[c];
}

// ---------------------------------------------------------------- rows kernel helpers
// One row of a C-column tile in LDS: C * sizeof(T) bytes as CPR 16-byte chunks.
template <class T, int C>
struct Tile {
  static constexpr int VPC = 16 / (int)sizeof(T);  // values per chunk
  static constexpr int CPR = C / VPC;              // chunks per row
  static constexpr int RB = C * (int)sizeof(T);    // bytes per row
  static_assert(CPR >= 1 && (CPR & (CPR - 1)) == 0, "tile width must be a power-of-two number of chunks");
  __device__ static __forceinline__ int at(int r, int k) { return r * RB + (k << 4); }
  __device__ static __forceinline__ int rot() { return (int)threadIdx.x & (CPR - 1); }  // first chunk of this lane
};

// Asynchronous copy of nrows rows (C values each, row stride ld) into the tile. Each lane
// moves one 16-byte chunk per instruction; the chunks of one wavefront land contiguously.
template <class T, int C>
__device__ __forceinline__ void stage_dma(char* lds, const T* src, int64_t ld, int nrows) {
  using L = Tile<T, C>;
  const int total = nrows * L::CPR;
  const int lane = threadIdx.x & 63;
  for (int s0 = threadIdx.x & ~63; s0 < total; s0 += blockDim.x) {
    const int s = s0 + lane;
    if (s < total) {
      const int r = s / L::CPR, k = s % L::CPR;
      __builtin_amdgcn_global_load_lds((const void*)(src + (int64_t)r * ld + k * L::VPC),
                                       (__attribute__((address_space(3))) void*)(lds + (s0 << 4)), 16, 0, 0);
    }
  }
}

// Synchronous copy into the same layout (partial or unaligned column tiles), zero beyond cvalid.
template <class T, int C>
__device__ __forceinline__ void stage_sync(char* lds, const T* src, int64_t ld, int nrows, int cvalid) {
  using L = Tile<T, C>;
  const int total = nrows * L::CPR;
  for (int s = threadIdx.x; s < total; s += blockDim.x) {
    const int r = s / L::CPR, k = s % L::CPR;
    T* d = reinterpret_cast<T*>(lds + L::at(r, k));
#pragma unroll
    for (int v = 0; v < L::VPC; v++) {
      const int c = k * L::VPC + v;
      d[v] = c < cvalid ? src[(int64_t)r * ld + c] : T(0);
    }
  }
}

// acc += coef * row r of the tile, accumulator slot t <- chunk (t + rot) mod CPR
template <class T, int C>
__device__ __forceinline__ void gather(T (&acc)[C], T coef, const char* lds, int r, int rot) {
  using L = Tile<T, C>;
  const char* row = lds + r * L::RB;
#pragma unroll
  for (int k = 0; k < L::CPR; k++) {
    const char* p = row + (((k + rot) & (L::CPR - 1)) << 4);
    if constexpr (sizeof(T) == 8) {
      const double2 v = *reinterpret_cast<const double2*>(p);
      acc[2 * k] += coef * v.x;
      acc[2 * k + 1] += coef * v.y;
    } else {
      const float4 v = *reinterpret_cast<const float4*>(p);
      acc[4 * k] += coef * v.x;
      acc[4 * k + 1] += coef * v.y;
      acc[4 * k + 2] += coef * v.z;
      acc[4 * k + 3] += coef * v.w;
    }
  }
}

// Load of a workgroup-uniform table entry through the constant address space, so the
// compiler issues a scalar load (counted apart from the vector loads and LDS DMA in flight).
template <class U>
__device__ __forceinline__ U ldu(const U* p, int64_t i) {
  return ((const __attribute__((address_space(4))) U*)(p))[i];
}

// Proton jumps of one target SD are stored per class, sorted by source row; a group is a
// run of jumps of one class with the same source row (several only for number operators).
// The groups of every SD are listed on the host as (class, first jump, end jump, source row);
// groups whose class has no source block in this product block are skipped.
struct GroupIt {
  int g, cls, jg, je, sb, p;  // cls == ncl: no group left
};

template <class T>
__device__ __forceinline__ GroupIt group_at(const HVArgs<T>& a, int b, int g, int gend) {
  for (; g < gend; g++) {
    const int* d = a.pg_desc + 4 * (int64_t)g;
    const int cls = ldu(d, 0);
    const int sb = ldu(a.src_blk, b * a.ncl + cls);
    if (sb >= 0) return {g, cls, ldu(d, 1), ldu(d, 2), sb, ldu(d, 3)};
  }
  return {gend, a.ncl, 0, 0, -1, 0};
}

constexpr int MAXE = 8;           // neutron jumps per (target, class) kept in registers
// MP targets per lane multiply the accumulators: MP > 1 is used for tile rows (C * sizeof(T), a
// power of two) of at most 128 / MP bytes, which is also all that a 72 KB buffer holds for
// sectors wider than (MP / 2) * 1024.
constexpr bool rows_mp_fits(size_t tile_row_bytes, int mp) { return tile_row_bytes * mp <= 128; }
// LDS rows of the class table used by the target's proton jumps (smaller with the 36 KB row
// buffers, so that two workgroups fit in the 160 KB of LDS of a CU)
constexpr int hs_bytes(int rbkb) { return rbkb == 36 ? 4096 : 8192; }

// Rows kernel: neutron-neutron and proton-neutron parts of W for one proton row p' of one
// block (App. B). One lane owns target n' (or MP of them; wider sectors are split in chunks) and the C
// columns of the tile. Its neutron jumps of the current class sit in registers; the class
// table rows of the proton ops sit in LDS; source rows stream through B0/B1.
// SB (one row buffer): the current source row is staged and waited for at every step; used
// for narrow sectors with wide source rows, where half the LDS lets two workgroups share a
// CU and overlap each other's staging instead of their own, and for the 144 KB buffer of the
// widest rows, where a wider column tile is worth more than the overlap.
// MP (targets per lane): sectors wider than 1024 give each lane MP targets n', n' + 1024, ...,
// so that a staged source row serves the whole sector instead of one 1024-wide chunk of it.
template <class T, int C, int NTB, int RBKB, bool DMA, bool SB = false, int MP = 1>
__global__ __launch_bounds__(NTB, (NTB == 768 && sizeof(T) == 4 && RBKB <= 36) ? 6 : 1) void hv_rows_kernel(HVArgs<T> a) {
  constexpr int MAXP = MP;  // targets per lane (sectors wider than MP * 1024 are split into chunks)
  // neutron jumps per (target, class) in registers: fewer with 4 targets per lane, fewest with
  // 32-byte tile rows (the rest are read from the table as they are used)
  constexpr int NE = MP >= 4 ? (C * (int)sizeof(T) >= 32 ? 2 : 4) : MAXE;
  constexpr int RBYTES = RBKB * 1024;
  constexpr int HSN = hs_bytes(RBKB) / (int)sizeof(T);
  __shared__ __align__(16) char B0[RBYTES];
  __shared__ __align__(16) char B1[SB ? 16 : RBYTES];
  __shared__ __align__(16) T HS[HSN];
  const int64_t nitems = a.bin_item0[a.bin_nblk];
  const int64_t item = xcd_item(blockIdx.x, nitems);
  if (item >= nitems) return;
  const int bi = find_block(a.bin_item0, a.bin_nblk, item);
  const int b = a.bin_blocks[bi];
  int64_t rel = item - a.bin_item0[bi];
  const int tc = (int)(rel % a.nchunk);
  rel /= a.nchunk;
  const int ct = (int)(rel % a.ntile);
  const int pl = (int)(rel / a.ntile);
  const int nthr = blockDim.x, tid = threadIdx.x;
  const int c0 = ct * C, cvalid = min(C, a.nb - c0);
  const int dn = a.blk_dn[b];
  const int64_t off = a.blk_off[b];
  const int gp = a.blk_p0[b] + pl;
  const int gn0 = a.blk_n0[b];
  const int tlo = tc * nthr * MAXP;
  if (tlo >= dn) return;  // chunk beyond this block's sector (bins mix sector widths)
  const int thi = min(dn, tlo + nthr * MAXP);
  const int ncl = a.ncl;
  const int rot = Tile<T, C>::rot();
  T acc[MAXP][C];
#pragma unroll
  for (int q = 0; q < MAXP; q++)
#pragma unroll
    for (int c = 0; c < C; c++) acc[q][c] = T(0);

  auto stage_row = [&](char* dst, int64_t row0, int rows) __attribute__((always_inline)) {
    const T* src = a.V + row0 * a.ldv + c0;
    if constexpr (DMA) stage_dma<T, C>(dst, src, a.ldv, rows);
    else stage_sync<T, C>(dst, src, a.ldv, rows, cvalid);
  };

  const int gend = ldu(a.pg_start, gp + 1);
  GroupIt it = group_at(a, b, ldu(a.pg_start, gp), gend);
  stage_row(B0, off + (int64_t)pl * dn, dn);
  if (!SB && it.cls < ncl) stage_row(B1, a.blk_off[it.sb] + (int64_t)it.p * a.blk_dn[it.sb], a.blk_dn[it.sb]);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();

  // own row: neutron-neutron part (single-particle energies included)
  const int ns0l = a.blk_nslice0[b];
#pragma unroll
  for (int q = 0; q < MAXP; q++) {
    const int n = tlo + q * nthr + tid;
    if (n < thi) {
      const int sl = ns0l + n / 64, ln = n % 64;
      const int base = a.ne_off[sl], wd = a.ne_w[sl];
      for (int k = 0; k < wd; k++) {
        const int at = base + k * 64 + ln;
        gather<T, C>(acc[q], a.ne_val[at], B0, a.ne_col[at], rot);
      }
    }
  }
  __syncthreads();

  // proton-neutron part
  int2 er[MAXP][NE];
  int eb[MAXP], ec[MAXP];
  int cur = -1, j0c = 0, hn = 0;
  bool hs_lds = false;
  const T* hg = a.h;
  auto step = [&](const char* rd, char* wr) __attribute__((always_inline)) {
    if (it.cls != cur) {  // new class: neutron jumps to registers, class-table rows to LDS
      cur = it.cls;
      const int cn = (2 * a.tjmax - cur / 2) * 2 + (cur & 1);
      const int* ns0 = a.nj_start + (int64_t)cn * (a.nn_total + 1) + gn0;
#pragma unroll
      for (int q = 0; q < MAXP; q++) {
        const int n = tlo + q * nthr + tid;
        eb[q] = n < thi ? ns0[n] : 0;
        ec[q] = n < thi ? ns0[n + 1] - eb[q] : 0;
#pragma unroll
        for (int i = 0; i < NE; i++) {
          er[q][i] = make_int2(0, 0);
          if (i < ec[q]) er[q][i] = a.nj_pack[eb[q] + i];
          // pin the loads here (before the barrier and the next DMA), not next to their first use
          asm volatile("" ::"v"(er[q][i].x), "v"(er[q][i].y));
        }
      }
      j0c = ldu(a.pj_start, gp * ncl + cur);
      const int nj = ldu(a.pj_start, gp * ncl + cur + 1) - j0c;
      hn = ldu(a.h_ncol, cur);
      hg = a.h + ldu(a.h_off, cur);
      hs_lds = nj * hn <= HSN;
      if (hs_lds)
        for (int e = tid; e < nj * hn; e += nthr) {
          const int jj = e / hn, o = e - jj * hn;
          HS[e] = hg[(a.pj_meta[j0c + jj] >> 1) * hn + o];
        }
      __builtin_amdgcn_s_waitcnt(0);  // entries in registers before any DMA is in flight
      __syncthreads();
    }
    const GroupIt nx = group_at(a, b, it.g + 1, gend);
    if constexpr (SB) {  // the only buffer is free (every lane passed the previous barrier)
      stage_row(B0, ldu(a.blk_off, it.sb) + (int64_t)it.p * ldu(a.blk_dn, it.sb), ldu(a.blk_dn, it.sb));
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
    } else if (nx.cls < ncl) {
      stage_row(wr, ldu(a.blk_off, nx.sb) + (int64_t)nx.p * ldu(a.blk_dn, nx.sb), ldu(a.blk_dn, nx.sb));
    }
    // hr points into LDS or into global memory: two copies of the loop keep every load
    // typed (a generic pointer would make the compiler wait for the DMA in flight).
    // Terms with the same source element are summed before the row is read: in the class of
    // zero change of M and parity (the diagonal class) every neutron SD's first nnum jumps are
    // its number operators (source n' itself), and a group of several proton jumps (the
    // number operators, source p') shares every neutron entry.
    const int nm = cur == 2 * a.tjmax ? a.nnum : 0;
    auto apply = [&](auto hrow) __attribute__((always_inline)) {
      auto body = [&](auto cf) __attribute__((always_inline)) {
#pragma unroll
        for (int q = 0; q < MAXP; q++) {
          if (nm > 0 && ec[q] >= nm) {
            T sum = T(0);
#pragma unroll
            for (int i = 0; i < NE; i++)
              if (i < nm) sum += cf(er[q][i]);
            gather<T, C>(acc[q], sum, rd, er[q][0].x, rot);
          }
#pragma unroll
          for (int i = 0; i < NE; i++)
            if (i >= nm && i < ec[q]) gather<T, C>(acc[q], cf(er[q][i]), rd, er[q][i].x, rot);
          // jumps beyond the register-held ones; with 16-byte tile rows (wide sectors, where most
          // jumps land here) four table loads are put in flight before their gathers
          int i = NE;
          if constexpr (C * sizeof(T) <= 16)
            for (; i + 4 <= ec[q]; i += 4) {
              int2 e[4];
#pragma unroll
              for (int u = 0; u < 4; u++) e[u] = a.nj_pack[eb[q] + i + u];
#pragma unroll
              for (int u = 0; u < 4; u++) gather<T, C>(acc[q], cf(e[u]), rd, e[u].x, rot);
            }
          for (; i < ec[q]; i++) {
            const int2 e = a.nj_pack[eb[q] + i];
            gather<T, C>(acc[q], cf(e), rd, e.x, rot);
          }
        }
      };
      if (it.je - it.jg == 1) {
        const int pm = ldu(a.pj_meta, it.jg);
        const auto hr = hrow(it.jg, pm);
        body([&](int2 e) __attribute__((always_inline)) {
          const T hv = hr[e.y >> 1];
          return ((e.y ^ pm) & 1) ? -hv : hv;
        });
      } else {
        body([&](int2 e) __attribute__((always_inline)) {
          T sum = T(0);
          for (int j = it.jg; j < it.je; j++) {
            const int pm = ldu(a.pj_meta, j);
            const T hv = hrow(j, pm)[e.y >> 1];
            sum += ((e.y ^ pm) & 1) ? -hv : hv;
          }
          return sum;
        });
      }
    };
    if (hs_lds)
      apply([&](int j, int) __attribute__((always_inline)) { return HS + (j - j0c) * hn; });
    else
      apply([&](int, int pm) __attribute__((always_inline)) { return hg + (pm >> 1) * hn; });
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    it = nx;
  };
  if constexpr (SB) {
    while (it.cls < ncl) step(B0, B0);
  } else {
    while (it.cls < ncl) {
      step(B1, B0);
      if (it.cls >= ncl) break;
      step(B0, B1);
    }
  }
  using L = Tile<T, C>;
#pragma unroll
  for (int q = 0; q < MAXP; q++) {
    const int n = tlo + q * nthr + tid;
    if (n < thi) {
      T* w = a.W + (off + (int64_t)pl * dn + n) * a.ldw + c0;
#pragma unroll
      for (int t = 0; t < L::CPR; t++) {
        const int k = (t + rot) & (L::CPR - 1);
#pragma unroll
        for (int v = 0; v < L::VPC; v++)
          if (k * L::VPC + v < cvalid) w[k * L::VPC + v] = acc[q][t * L::VPC + v];
      }
    }
  }
}

// Columns kernel: proton-proton part, W[:, n] += Hpp V[:, n] for one neutron column n of one
// block; the column (all proton rows of the block, one column tile) is staged in LDS and one
// lane owns one target proton row p'.
template <class T, int C, int MAXP>
__global__ __launch_bounds__(1024) void hv_cols_kernel(HVArgs<T> a) {
  extern __shared__ __align__(16) char smem_[];
  constexpr int RS = row_stride<T, C>();
  T* colv = reinterpret_cast<T*>(smem_);
  const int64_t nitems = a.citem0[a.nblocks];
  const int64_t item = xcd_item(blockIdx.x, nitems);
  if (item >= nitems) return;
  const int b = find_block(a.citem0, a.nblocks, item);
  int64_t rel = item - a.citem0[b];
  const int tc = (int)(rel % a.nchunk);
  rel /= a.nchunk;
  const int ct = (int)(rel % a.ntile);
  const int n = (int)(rel / a.ntile);
  const int nthr = blockDim.x, tid = threadIdx.x;
  const int c0 = ct * C, cvalid = min(C, a.nb - c0);
  const int dn = a.blk_dn[b], dp = a.blk_dp[b];
  const int64_t off = a.blk_off[b];
  stage<T, C>(colv, a.V + (off + n) * a.ldv + c0, (int64_t)dn * a.ldv, dp, cvalid);
  __syncthreads();
  const int tlo = tc * nthr * MAXP;
#pragma unroll
  for (int q = 0; q < MAXP; q++) {
    const int p = tlo + q * nthr + tid;
    if (p < dp) {
      T acc[C];
#pragma unroll
      for (int c = 0; c < C; c++) acc[c] = T(0);
      const int sl = a.blk_pslice0[b] + p / 64, ln = p % 64;
      const int base = a.pe_off[sl], wd = a.pe_w[sl];
      for (int k = 0; k < wd; k++) {
        const int at = base + k * 64 + ln;
        axpy_row<T, C>(acc, a.pe_val[at], colv + a.pe_col[at] * RS);
      }
      T* w = a.W + (off + (int64_t)p * dn + n) * a.ldw + c0;
#pragma unroll
      for (int c = 0; c < C; c++)
        if (c < cvalid) w[c] += acc[c];
    }
  }
}

template <class T, int C, int NTB, int RB, int MP = 1>
static void launch_rows(const HVArgs<T>& a, const HVBin& B, hipStream_t s) {
  const dim3 grid((unsigned)((B.items + 7) / 8 * 8)), block(B.nthr);
  constexpr bool SB = NTB == 256 || RB == 144;  // one buffer: narrow sectors, or the widest rows
  if (a.dma) hipLaunchKernelGGL((hv_rows_kernel<T, C, NTB, RB, true, SB, MP>), grid, block, 0, s, a);
  else hipLaunchKernelGGL((hv_rows_kernel<T, C, NTB, RB, false, SB, MP>), grid, block, 0, s, a);
}
template <class T, int C, int MP>
static void launch_cols(const HVArgs<T>& a, const HVPlan& P, hipStream_t s) {
  hipLaunchKernelGGL((hv_cols_kernel<T, C, MP>), dim3((unsigned)((P.cols_items + 7) / 8 * 8)), dim3(P.nthr_c),
                     P.shm_c, s, a);
}

template <class T, int CC>
static void dispatch_cols(HVArgs<T>& a, const HVPlan& P, hipStream_t s) {
  if (P.maxp_c == 1) launch_cols<T, CC, 1>(a, P, s);
  else if (P.maxp_c == 2) launch_cols<T, CC, 2>(a, P, s);
  else launch_cols<T, CC, 4>(a, P, s);
}

template <class T, int C>
static void dispatch_c(HVArgs<T>& a, const HVPlan& P, hipStream_t s) {
  for (const auto& Bp : P.bins) {
    const HVBin& B = *Bp;
    a.nchunk = B.nchunk;
    a.bin_blocks = B.blocks.as<int>();
    a.bin_item0 = B.item0.as<int64_t>();
    a.bin_nblk = B.nblk;
#define TRBL_ROWS_RB(NTB)                                                   \
  (B.rb_kb == 24   ? launch_rows<T, C, NTB, 24>(a, B, s)                    \
   : B.rb_kb == 36 ? launch_rows<T, C, NTB, 36>(a, B, s)                    \
   : B.rb_kb == 72 ? launch_rows<T, C, NTB, 72>(a, B, s)                    \
                   : launch_rows<T, C, NTB, 144>(a, B, s))
    if (B.ntb == 256) TRBL_ROWS_RB(256);
    else if (B.ntb == 768) TRBL_ROWS_RB(768);
    else if (B.mp == 4) {
      if constexpr (rows_mp_fits(C * sizeof(T), 4)) {
        if (B.rb_kb == 144) launch_rows<T, C, 1024, 144, 4>(a, B, s);
        else launch_rows<T, C, 1024, 72, 4>(a, B, s);
      } else TRBL_REQUIRE(false, TRBL_E_INVALID, "targets-per-lane plan does not match the column tile");
    } else if (B.mp == 2) {
      if constexpr (rows_mp_fits(C * sizeof(T), 2)) {
        if (B.rb_kb == 144) launch_rows<T, C, 1024, 144, 2>(a, B, s);
        else launch_rows<T, C, 1024, 72, 2>(a, B, s);
      } else TRBL_REQUIRE(false, TRBL_E_INVALID, "targets-per-lane plan does not match the column tile");
    } else TRBL_ROWS_RB(1024);
#undef TRBL_ROWS_RB
  }
  a.nchunk = P.nchunk_c;
  a.ntile = P.ntile_c;
  if (P.Cc == C) dispatch_cols<T, C>(a, P, s);
  else if (P.Cc * 2 == C) {
    if constexpr (C / 2 >= 16 / (int)sizeof(T)) dispatch_cols<T, C / 2>(a, P, s);
  } else {
    if constexpr (C / 4 >= 16 / (int)sizeof(T)) dispatch_cols<T, C / 4>(a, P, s);
  }
  a.ntile = P.ntile;
}

// All launches of one block H.V (rows kernel per bin, then the columns kernel).
template <class T>
void dispatch_hv(HVArgs<T>& a, const HVPlan& P, hipStream_t s) {
  if constexpr (sizeof(T) == 8) {
    switch (P.C) {
      case 2: dispatch_c<T, 2>(a, P, s); break;
      case 4: dispatch_c<T, 4>(a, P, s); break;
      case 8: dispatch_c<T, 8>(a, P, s); break;
      default: dispatch_c<T, 16>(a, P, s); break;
    }
  } else {
    switch (P.C) {
      case 4: dispatch_c<T, 4>(a, P, s); break;
      case 8: dispatch_c<T, 8>(a, P, s); break;
      case 16: dispatch_c<T, 16>(a, P, s); break;
      default: dispatch_c<T, 32>(a, P, s); break;
    }
  }
}

}  // namespace trbl
