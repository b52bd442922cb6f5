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
// gfx950 (no registers involved). Rows are stored plainly. A 16-byte LDS read
// of a wavefront is served half a wavefront at a time, at two lanes per
// 16-byte position of the 256-byte bank window when no position is shared by
// more: lane l reads chunk t ^ (l mod chunks-per-row) of its row at step t
// (accumulator slot t holds that chunk, which the final store undoes), and the
// host orders each lane's neutron jumps so that the rows of the lanes reading
// one chunk position fall in different parts of the window.
#pragma once
#include <type_traits>

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
  int own;               // identical-particle parts only (the pn part is added by the pair blocks)
  int zs;                // own-row kernel: slots of the pair-block buffer summed into W (0: none)
  int ppset;             // columns kernel writes W (instead of adding to it); the own-row kernel then adds
  int64_t zstride;       // elements between slots of that buffer ([slot][D][16] values of type T)
  const void* zbuf;
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
  const uint32_t* nj32;  // the same jumps packed: sign << 31 | op << 16 | source local index
  const int* pg_cend;    // per jump group: first group after the run of its class
  const int* nlane;      // lane order of the rows kernel: sector-local neutron SD of each lane
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
  __device__ static __forceinline__ int rot() { return (int)threadIdx.x & (CPR - 1); }  // chunk order of this lane
  // rows per 256-byte LDS bank window, and so the zero rows kept (one per part of the window)
  static constexpr int NZ = RB >= 256 ? 1 : 256 / RB;
};

// The part of the bank window (source row mod 16, lowest bit most significant) that the lane
// at position l of its sector prefers; the neutron jump lists are ordered for it on the host.
__device__ __forceinline__ int bank_pref(int l) {
  return ((l & 1) << 3) | ((l & 2) << 1) | ((l & 4) >> 1) | ((l & 8) >> 3);
}

// Asynchronous copy of nrows rows (C values each, row stride ld) into the tile by the
// global->LDS DMA of buffer loads: each lane moves one 16-byte chunk per instruction and the
// chunks of one wavefront land contiguously. The row base is a buffer descriptor, the
// wavefront's position a scalar offset and the lane's position a register that never changes,
// so nothing the DMA reads is overwritten while it is in flight (out-of-range offsets read 0).
template <class T, int C>
__device__ __forceinline__ void stage_dma(char* lds, const T* src, int64_t ld, int nrows) {
#if defined(__HIP_DEVICE_COMPILE__)  // buffer descriptors exist only in the device pass
  using L = Tile<T, C>;
  const int total = nrows * L::CPR;
  const int lane = threadIdx.x & 63;
  const int rowb = (int)(ld * (int64_t)sizeof(T));
  const int voff = (lane / L::CPR) * rowb + (lane % L::CPR) * 16;
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void*)src, (short)0, 0x7fffffff, 0x00020000);
  const int w0 = __builtin_amdgcn_readfirstlane((int)threadIdx.x & ~63);
  const int wstep = __builtin_amdgcn_readfirstlane((int)blockDim.x);
  for (int s0 = w0; s0 < total; s0 += wstep)
    if (s0 + lane < total)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void*)(lds + (s0 << 4)), 16, voff,
                                               (s0 / L::CPR) * rowb, 0, 0);
#endif
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

// Neutron jumps as the rows kernel reads them: one word per jump, sign in bit 31, operator
// index inside its class in bits 16..30, source index inside its sector in bits 0..15.
constexpr uint32_t NJ_SIGN = 0x80000000u;
__device__ __forceinline__ int nj_src(uint32_t e) { return (int)(e & 0xFFFFu); }
__device__ __forceinline__ int nj_op(uint32_t e) { return (int)((e >> 16) & 0x7FFFu); }
// h with the jump's sign applied by flipping the sign bit
__device__ __forceinline__ double signed_coef(double h, uint32_t e) {
  return __hiloint2double(__double2hiint(h) ^ (int)(e & NJ_SIGN), __double2loint(h));
}
__device__ __forceinline__ float signed_coef(float h, uint32_t e) {
  return __int_as_float(__float_as_int(h) ^ (int)(e & NJ_SIGN));
}

// MP targets per lane multiply the accumulators: MP > 1 is used for tile rows (C * sizeof(T), a
// power of two) of at most 128 / MP bytes, which is also all that a 72 KB buffer holds for
// sectors wider than (MP / 2) * 1024.
constexpr bool rows_mp_fits(size_t tile_row_bytes, int mp) { return tile_row_bytes * mp <= 128; }
// LDS bytes of the coefficient rows next to the row buffers: 16 KB where the buffers take 144 KB
// (one workgroup per CU), else 8 KB (so that two workgroups of 72 KB buffers share a CU)
constexpr int hs_bytes(int rbkb, bool sb) { return (sb ? rbkb : 2 * rbkb) >= 144 ? 16384 : 8192; }

// acc += coef * row of the tile at `row`: the CPR chunk loads are issued together, then the FMAs.
// Accumulator slot t holds chunk t ^ rot (rot = lane mod CPR), so that the lanes of a wavefront
// reading random rows start on different LDS banks; since rows are CPR * 16 bytes and aligned,
// the address of chunk t ^ rot is (row + rot * 16) ^ (t * 16).
template <class T>
using RowChunk = typename std::conditional<sizeof(T) == 8, double2, float4>::type;
template <class T, int C>
__device__ __forceinline__ void load_row(RowChunk<T>* v, const char* lds, int row_byte) {
  using L = Tile<T, C>;
  const int a0 = row_byte + (L::rot() << 4);
#pragma unroll
  for (int t = 0; t < L::CPR; t++) v[t] = *reinterpret_cast<const RowChunk<T>*>(lds + (a0 ^ (t << 4)));
}
template <class T, int C>
__device__ __forceinline__ void fma_row(T (&acc)[C], T coef, const RowChunk<T>* v) {
  using L = Tile<T, C>;
#pragma unroll
  for (int t = 0; t < L::CPR; t++) {
    if constexpr (sizeof(T) == 8) {
      acc[2 * t] += coef * v[t].x;
      acc[2 * t + 1] += coef * v[t].y;
    } else {
      acc[4 * t] += coef * v[t].x;
      acc[4 * t + 1] += coef * v[t].y;
      acc[4 * t + 2] += coef * v[t].z;
      acc[4 * t + 3] += coef * v[t].w;
    }
  }
}
template <class T, int C>
__device__ __forceinline__ void gather_row(T (&acc)[C], T coef, const char* lds, int row_byte) {
  RowChunk<T> v[Tile<T, C>::CPR];
  load_row<T, C>(v, lds, row_byte);
  fma_row<T, C>(acc, coef, v);
}

// Rows kernel: neutron-neutron and proton-neutron parts of W for one proton row p' of one
// block (App. B). One lane owns one target n' (or MP of them: lanes l, l + width, ...) and the
// C columns of the tile; lane l of a sector serves the SD nlane[sector start + l], an order in
// which neighbouring lanes have similar numbers of jumps per class.
//
// The proton jumps of p' are walked as groups (one source row p each, several jumps only for
// the proton number operators), class by class. Per class, each lane holds its neutron jumps
// of the opposite class in registers, and LDS holds one coefficient row per group: the proton
// signs and the jumps of a group summed into HS[group][op_n] = sum_j s_j h[op_p(j)][op_n].
// A step (one group, one source row) then costs, per element, one LDS read of the coefficient
// and CPR 16-byte LDS reads of the source row, and nothing else: the compute phase issues no
// global or scalar loads, so the asynchronous copy of the next source row (global->LDS DMA
// into the other buffer) stays in flight until the closing barrier.
//
// With one target per lane every lane runs as many elements as the longest jump list of its
// wavefront; shorter lists are padded with a jump to row Z of the buffer, a row of zeros that
// no copy overwrites, so the element loop has no divergent branches (and, with the lane order
// above, little padding). In the class of no change of M and
// parity each neutron SD's number operators (source n' itself) are summed into one element.
// SB (one row buffer): the current source row is staged and waited for at every step; used
// for narrow sectors, where half the LDS lets two workgroups share a CU and overlap each
// other's staging, and for the 144 KB buffer of the widest rows.
template <class T, int C, int NTB, int RBKB, bool DMA, bool SB = false, int MP = 1, int NR = 16>
__global__ __launch_bounds__(NTB) void hv_rows_kernel(HVArgs<T> a) {
  using L = Tile<T, C>;
  constexpr int RBYTES = RBKB * 1024;
  constexpr int HSN = hs_bytes(RBKB, SB) / (int)sizeof(T);
  constexpr int ZBASE = RBYTES / L::RB - L::NZ;  // the zero rows of each buffer: ZBASE .. ZBASE + NZ - 1
  static_assert(ZBASE + L::NZ - 1 < 65536, "row index must fit the packed jumps");
  __shared__ __align__(256) char B0[RBYTES];
  __shared__ __align__(256) char B1[SB ? 16 : RBYTES];
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
  const int tlo = tc * nthr * MP;
  if (tlo >= dn) return;  // chunk beyond this block's sector (bins mix sector widths)
  const int thi = min(dn, tlo + nthr * MP);
  const int ncl = a.ncl;
  int tg[MP];  // this lane's targets (sector-local neutron index), -1 for none
#pragma unroll
  for (int q = 0; q < MP; q++) {
    const int ln = tlo + q * nthr + tid;
    tg[q] = ln < thi ? a.nlane[gn0 + ln] : -1;
  }
  T acc[MP][C];
#pragma unroll
  for (int q = 0; q < MP; q++)
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
  for (int k = tid; k < L::NZ * L::CPR; k += nthr) {  // the zero rows (above every staged row)
    *reinterpret_cast<float4*>(B0 + ZBASE * L::RB + (k << 4)) = make_float4(0.f, 0.f, 0.f, 0.f);
    if constexpr (!SB) *reinterpret_cast<float4*>(B1 + ZBASE * L::RB + (k << 4)) = make_float4(0.f, 0.f, 0.f, 0.f);
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();

  // own row: neutron-neutron part (single-particle energies included), sliced ELL entries read
  // four at a time
  const int ns0l = a.blk_nslice0[b];
#pragma unroll
  for (int q = 0; q < MP; q++) {
    const int ln = tlo + q * nthr + tid;
    if (ln < thi) {
      const int sl = ns0l + ln / 64, lo = ln % 64;
      const int base = a.ne_off[sl], wd = a.ne_w[sl];
      for (int k = 0; k < wd; k += 4) {
        int cc[4];
        T vv[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
          const int at = base + (k + u) * 64 + lo;
          cc[u] = k + u < wd ? a.ne_col[at] : 0;
          vv[u] = k + u < wd ? a.ne_val[at] : T(0);
        }
#pragma unroll
        for (int u = 0; u < 4; u++) gather_row<T, C>(acc[q], vv[u], B0, cc[u] * L::RB);
      }
    }
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();

  // proton-neutron part
  // padding jump: operator 0, the zero row in the lane's preferred part of the bank window
  const uint32_t zj = (uint32_t)(ZBASE + (bank_pref(tid) & (L::NZ - 1)));
  const int dcls = 2 * a.tjmax;        // class of no change of M and parity
  uint32_t er[MP][NR];
  int eb[MP], ec[MP];
  uint32_t e0[MP];  // first element: a jump, or (number-operator class) the own row
  uint32_t nmo[MP][4];  // number-operator columns of the coefficient rows, two 16-bit fields a word
  int nm = 0, ecm = 0;
  int cur = -1, hs_g0 = 0, hs_gn = 0, hn = 1;
  // class change: this lane's neutron jumps of the opposite class into registers
  auto load_class = [&](int cls) __attribute__((always_inline)) {
    cur = cls;
    nm = (cls == dcls) ? a.nnum : 0;
    const int cn = (2 * a.tjmax - cls / 2) * 2 + (cls & 1);
    const int* ns0 = a.nj_start + (int64_t)cn * (a.nn_total + 1) + gn0;
    int emax = 0;
#pragma unroll
    for (int q = 0; q < MP; q++) {
      // loads are unconditional (every index is valid: lanes without a target read entry 0,
      // and the table is padded by 32 entries) and pinned here, before the DMA of the step:
      // a load left for the compiler to sink into the compute phase would make it wait there
      const int n = tg[q];
      const int ja = ns0[max(n, 0)], jb = ns0[max(n, 0) + 1];
      const int j0 = n >= 0 ? ja : 0;
      const int cnt = n >= 0 ? jb - ja : 0;
      if constexpr (MP == 1) {
        // element 0: the merged number operators (row n'), else the first jump; the rest after it
        const int skip = nm > 0 ? nm : 1;
        uint32_t f[8];
#pragma unroll
        for (int k = 0; k < 8; k++) f[k] = a.nj32[j0 + k];
        e0[q] = n < 0 ? zj : nm > 0 ? (uint32_t)n : (cnt > 0 ? f[0] : zj);
#pragma unroll
        for (int k = 0; k < 4; k++)
          nmo[q][k] = n >= 0 ? (uint32_t)nj_op(f[2 * k]) | ((uint32_t)nj_op(f[2 * k + 1]) << 16) : 0u;
        eb[q] = j0 + skip;
        ec[q] = max(cnt - skip, 0);
#pragma unroll
        for (int i = 0; i < NR; i++) {
          const uint32_t e = a.nj32[eb[q] + i];
          er[q][i] = i < ec[q] ? e : zj;
        }
        asm volatile("" ::"v"(e0[q]));
#pragma unroll
        for (int k = 0; k < 4; k++) asm volatile("" ::"v"(nmo[q][k]));
      } else {
        eb[q] = j0;
        ec[q] = cnt;
#pragma unroll
        for (int i = 0; i < NR; i++) er[q][i] = a.nj32[eb[q] + i];
      }
#pragma unroll
      for (int i = 0; i < NR; i++) asm volatile("" ::"v"(er[q][i]));
      emax = max(emax, ec[q]);
    }
    // longest list of the wavefront (uniform)
    ecm = 0;
#pragma unroll
    for (int i = 0; i < NR; i++)
      if (__builtin_amdgcn_ballot_w64(emax > i) != 0) ecm = i + 1;
    hn = ldu(a.h_ncol, cls);
  };
  // coefficient rows of the groups g0 .. (end of the class run, or as many as HS holds)
  auto load_hs = [&](int g0) __attribute__((always_inline)) {
    const int cend = ldu(a.pg_cend, g0);
    hs_g0 = g0;
    hs_gn = min(cend - g0, HSN / hn);
    const T* hg = a.h + ldu(a.h_off, cur);
    for (int e = tid; e < hs_gn * hn; e += nthr) {
      const int gl = e / hn, o = e - gl * hn;
      const int* d = a.pg_desc + 4 * (int64_t)(g0 + gl);
      T sum = T(0);
      for (int j = d[1]; j < d[2]; j++) {
        const int pm = a.pj_meta[j];
        const T hv = hg[(pm >> 1) * hn + o];
        sum += (pm & 1) ? -hv : hv;
      }
      HS[e] = sum;
    }
  };
  auto step = [&](const char* rd, char* wr) __attribute__((always_inline)) {
    if (it.cls != cur || it.g >= hs_g0 + hs_gn) {
      if (it.cls != cur) {
        load_class(it.cls);
        // also here, so that no path the compiler makes around the barrier below carries these
        // loads into the compute phase (a wait for them there would also wait for the DMA)
        __builtin_amdgcn_s_waitcnt(0);
      }
      load_hs(it.g);
      __builtin_amdgcn_s_waitcnt(0);  // jumps in registers, HS written, before any DMA is in flight
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
    const T* hrow = HS + (it.g - hs_g0) * hn;
    auto coef = [&](uint32_t e) __attribute__((always_inline)) { return signed_coef(hrow[nj_op(e)], e); };
    auto rowb = [&](uint32_t e) __attribute__((always_inline)) { return nj_src(e) * L::RB; };
    if constexpr (MP == 1) {
      RowChunk<T> buf[1][L::CPR];
      T cf[1];
      // element 0
      if (nm > 0) {
        T sum = T(0);
#pragma unroll
        for (int k = 0; k < 8; k++)
          if (k < nm) sum += hrow[(nmo[0][k >> 1] >> (16 * (k & 1))) & 0xFFFFu];  // number operators carry no sign
        cf[0] = sum;
        load_row<T, C>(buf[0], rd, (int)(e0[0] & 0xFFFFu) * L::RB);
      } else {
        cf[0] = coef(e0[0]);
        load_row<T, C>(buf[0], rd, rowb(e0[0]));
      }
      fma_row<T, C>(acc[0], cf[0], buf[0]);
      // elements 1 .. ecm (uniform trip count: padded lists, no divergent branches)
#pragma unroll
      for (int i = 0; i < NR; i++)
        if (i < ecm) gather_row<T, C>(acc[0], coef(er[0][i]), rd, rowb(er[0][i]));
    } else {
#pragma unroll
      for (int q = 0; q < MP; q++) {
        if (tg[q] < 0) continue;
        if (nm > 0) {
          T sum = T(0);
#pragma unroll
          for (int i = 0; i < NR; i++)
            if (i < nm) sum += coef(er[q][i]);
          gather_row<T, C>(acc[q], sum, rd, rowb(er[q][0]));
        }
#pragma unroll
        for (int i = 0; i < NR; i++)
          if (i >= nm && i < ec[q]) gather_row<T, C>(acc[q], coef(er[q][i]), rd, rowb(er[q][i]));
        // jumps beyond the register-held ones, read from the table
        for (int i = NR; i < ec[q]; i++) {
          const uint32_t e = a.nj32[eb[q] + i];
          gather_row<T, C>(acc[q], coef(e), rd, rowb(e));
        }
      }
    }
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
#pragma unroll
  for (int q = 0; q < MP; q++) {
    if (tg[q] >= 0) {
      T* w = a.W + (off + (int64_t)pl * dn + tg[q]) * a.ldw + c0;
#pragma unroll
      for (int t = 0; t < L::CPR; t++) {
        const int k = t ^ L::rot();
#pragma unroll
        for (int v = 0; v < L::VPC; v++)
          if (k * L::VPC + v < cvalid) w[k * L::VPC + v] = acc[q][t * L::VPC + v];
      }
    }
  }
}

// Own-row kernel: the neutron-neutron part and the diagonal of the rows kernel without its pn part,
// for products whose pn part comes from the pair blocks. One workgroup per target proton row
// (and column tile); the row is staged once in LDS (dynamic size: the widest sector of the bin).
template <class T, int C, int NTB, bool DMA>
__global__ __launch_bounds__(NTB) void hv_own_kernel(HVArgs<T> a) {
  using L = Tile<T, C>;
  extern __shared__ __align__(256) char B0[];
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
  const int gn0 = a.blk_n0[b];
  const int tlo = tc * nthr;
  if (tlo >= dn) return;
  const T* src = a.V + (off + (int64_t)pl * dn) * a.ldv + c0;
  if constexpr (DMA) stage_dma<T, C>(B0, src, a.ldv, dn);
  else stage_sync<T, C>(B0, src, a.ldv, dn, cvalid);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  const int ln = tlo + tid;
  const bool live = ln < dn;
  T acc[C];
#pragma unroll
  for (int c = 0; c < C; c++) acc[c] = T(0);
  const int sl = a.blk_nslice0[b] + min(ln, dn - 1) / 64, lo = ln % 64;
  const int base = a.ne_off[sl], wd = live ? a.ne_w[sl] : 0;
  for (int k = 0; k < wd; k += 4) {
    int cc[4];
    T vv[4];
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const int at = base + (k + u) * 64 + lo;
      cc[u] = k + u < wd ? a.ne_col[at] : 0;
      vv[u] = k + u < wd ? a.ne_val[at] : T(0);
    }
#pragma unroll
    for (int u = 0; u < 4; u++) gather_row<T, C>(acc, vv[u], B0, cc[u] * L::RB);
  }
  if constexpr (C == 16) {
    if (a.zs > 0) {
      // the pn part from the pair-block slots: park the rows in LDS (target order), then stream the
      // slots of the proton row's dn targets in address order and write W once
      __syncthreads();  // every lane has read its staged source rows
      if (live) {
        const int tg = a.nlane[gn0 + ln];
#pragma unroll
        for (int t = 0; t < L::CPR; t++) {
          T* d = reinterpret_cast<T*>(B0 + L::at(tg, t ^ L::rot()));
#pragma unroll
          for (int v = 0; v < L::VPC; v++) d[v] = acc[t * L::VPC + v];
        }
      }
      __syncthreads();
      typedef T zv __attribute__((ext_vector_type(L::VPC)));  // one 16-byte chunk
      const int64_t r0 = off + (int64_t)pl * dn;
      const int lo_t = tlo, hi_t = min(dn, tlo + nthr);
      for (int e = lo_t * L::CPR + tid; e < hi_t * L::CPR; e += nthr) {
        const int t = e / L::CPR, k = e % L::CPR;
        zv v = *reinterpret_cast<const zv*>(B0 + L::at(t, k));
        const T* z = static_cast<const T*>(a.zbuf) + (r0 + t) * 16 + L::VPC * k;
        int q = 0;
        for (; q + 8 <= a.zs; q += 8) {  // eight slots in flight, summed in slot order
          zv zq[8];
#pragma unroll
          for (int j = 0; j < 8; j++) zq[j] = __builtin_nontemporal_load(reinterpret_cast<const zv*>(z + (q + j) * a.zstride));
#pragma unroll
          for (int j = 0; j < 8; j++) v += zq[j];
        }
        for (; q < a.zs; q++) v += __builtin_nontemporal_load(reinterpret_cast<const zv*>(z + q * a.zstride));
        T* w = a.W + (r0 + t) * a.ldw + c0 + L::VPC * k;
#pragma unroll
        for (int j = 0; j < L::VPC; j++)
          if (L::VPC * k + j < cvalid) w[j] = a.ppset ? w[j] + v[j] : v[j];
      }
      return;
    }
  }
  if (!live) return;
  T* w = a.W + (off + (int64_t)pl * dn + a.nlane[gn0 + ln]) * a.ldw + c0;
#pragma unroll
  for (int t = 0; t < L::CPR; t++) {
    const int k = t ^ L::rot();
#pragma unroll
    for (int v = 0; v < L::VPC; v++)
      if (k * L::VPC + v < cvalid) w[k * L::VPC + v] = a.ppset ? w[k * L::VPC + v] + acc[t * L::VPC + v] : acc[t * L::VPC + v];
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
      if (a.ppset) {
#pragma unroll
        for (int c = 0; c < C; c++)
          if (c < cvalid) w[c] = acc[c];
      } else {
#pragma unroll
        for (int c = 0; c < C; c++)
          if (c < cvalid) w[c] += acc[c];
      }
    }
  }
}

template <class T, int C, int NTB, int RB, int MP = 1>
static void launch_rows(const HVArgs<T>& a, const HVBin& B, hipStream_t s) {
  const dim3 grid((unsigned)((B.items + 7) / 8 * 8)), block(B.nthr);
  constexpr bool SB = NTB == 256 || RB == 144;  // one buffer: narrow sectors, or the widest rows
  // the copy variant is a template parameter: a kernel that can take either path makes the
  // compiler wait for the DMA in flight before every LDS read
  if constexpr (MP == 1) {
    if (B.nr == 32) {
      if (a.dma) hipLaunchKernelGGL((hv_rows_kernel<T, C, NTB, RB, true, SB, MP, 32>), grid, block, 0, s, a);
      else hipLaunchKernelGGL((hv_rows_kernel<T, C, NTB, RB, false, SB, MP, 32>), grid, block, 0, s, a);
    } else {
      if (a.dma) hipLaunchKernelGGL((hv_rows_kernel<T, C, NTB, RB, true, SB, MP, 16>), grid, block, 0, s, a);
      else hipLaunchKernelGGL((hv_rows_kernel<T, C, NTB, RB, false, SB, MP, 16>), grid, block, 0, s, a);
    }
  } else {
    if (a.dma) hipLaunchKernelGGL((hv_rows_kernel<T, C, NTB, RB, true, SB, MP, 8>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((hv_rows_kernel<T, C, NTB, RB, false, SB, MP, 8>), grid, block, 0, s, a);
  }
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

template <class T, int C, int NTB>
static void launch_own(const HVArgs<T>& a, const HVBin& B, hipStream_t s) {
  const dim3 grid((unsigned)((B.items + 7) / 8 * 8)), block(B.nthr);
  const size_t shm = (size_t)B.maxdn * C * sizeof(T);
  if (a.dma) hipLaunchKernelGGL((hv_own_kernel<T, C, NTB, true>), grid, block, shm, s, a);
  else hipLaunchKernelGGL((hv_own_kernel<T, C, NTB, false>), grid, block, shm, s, a);
}

template <class T, int C>
static void dispatch_c(HVArgs<T>& a, const HVPlan& P, hipStream_t s, int parts, unsigned binmask) {
  for (size_t bi = 0; bi < P.bins.size(); bi++) {
    if (!(parts & 1)) break;
    if (!((binmask >> bi) & 1)) continue;
    const HVBin& B = *P.bins[bi];
    a.nchunk = B.nchunk;
    a.bin_blocks = B.blocks.as<int>();
    a.bin_item0 = B.item0.as<int64_t>();
    a.bin_nblk = B.nblk;
    if (a.own) {
      TRBL_REQUIRE(B.mp == 1, TRBL_E_INVALID, "own-row plan with several targets per lane");
      if (B.ntb == 256) launch_own<T, C, 256>(a, B, s);
      else if (B.ntb == 768) launch_own<T, C, 768>(a, B, s);
      else launch_own<T, C, 1024>(a, B, s);
      continue;
    }
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
  if (!(parts & 2)) return;
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

// Launches of one block H.V: parts 1 = the rows (or own-row) kernel per bin, 2 = the columns kernel.
template <class T>
void dispatch_hv(HVArgs<T>& a, const HVPlan& P, hipStream_t s, int parts, unsigned binmask) {
  if constexpr (sizeof(T) == 8) {
    switch (P.C) {
      case 2: dispatch_c<T, 2>(a, P, s, parts, binmask); break;
      case 4: dispatch_c<T, 4>(a, P, s, parts, binmask); break;
      case 8: dispatch_c<T, 8>(a, P, s, parts, binmask); break;
      default: dispatch_c<T, 16>(a, P, s, parts, binmask); break;
    }
  } else {
    switch (P.C) {
      case 4: dispatch_c<T, 4>(a, P, s, parts, binmask); break;
      case 8: dispatch_c<T, 8>(a, P, s, parts, binmask); break;
      case 16: dispatch_c<T, 16>(a, P, s, parts, binmask); break;
      default: dispatch_c<T, 32>(a, P, s, parts, binmask); break;
    }
  }
}

}  // namespace trbl
