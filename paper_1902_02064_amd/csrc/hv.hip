// On-the-fly block H.V (App. B) and device-side basis indexing (App. A).
//
// W = H V for nb vectors stored row-major [D][ld]. Every output row
// (p', n') of a proton-major block b' is produced by one lane group:
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
// across the nb vectors held by the nb lanes of the group.
#include "internal.h"

namespace trbl {

template <class T>
struct HVArgs {
  const T* V;
  T* W;
  int64_t ldv, ldw;
  int nb, ncl, tjmax, nblocks;
  int C, ntile, nchunk;  // column tile width, column tiles, target chunks per row/column
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
  const int* nj_start;  // class-major: [cls * (nn_total + 1) + g]
  const int2* nj_pack;  // (source local index, op << 1 | sign)
  const int* h_off;
  const int* h_ncol;
  const T* h;
  const int* pp_ptr;
  const int* pp_col;
  const T* pp_val;
  const int* nn_ptr;
  const int* nn_col;
  const T* nn_val;
  const int* pe_off;   // sliced-ELL identical-particle operators (proton, neutron)
  const int* pe_w;
  const int* pe_col;
  const T* pe_val;
  const int* ne_off;
  const int* ne_w;
  const int* ne_col;
  const T* ne_val;
  const int* blk_pslice0;
  const int* blk_nslice0;
  const int64_t* item0;  // per block: first work item (rows kernel), size nblocks + 1
  const int64_t* citem0; // per block: first work item (columns kernel)
  size_t row_bytes, ent_bytes, hs_bytes;  // dynamic LDS partition of the rows kernel
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

// register prefetch of a row slab (issued early, written to LDS after a barrier)
constexpr int MAXPF = 16;
template <class T, int C>
__device__ __forceinline__ void prefetch(T (&pf)[MAXPF], const T* src, int64_t rstride, int nrows, int cvalid) {
  const int n = nrows * C;
#pragma unroll
  for (int i = 0; i < MAXPF; i++) {
    const int e = threadIdx.x + i * blockDim.x;
    if (e < n) {
      const int r = e / C, c = e % C;
      pf[i] = (c < cvalid) ? src[(int64_t)r * rstride + c] : T(0);
    }
  }
}
template <class T, int C>
__device__ __forceinline__ void commit(T* lds, const T (&pf)[MAXPF], int nrows) {
  constexpr int RS = row_stride<T, C>();
  const int n = nrows * C;
#pragma unroll
  for (int i = 0; i < MAXPF; i++) {
    const int e = threadIdx.x + i * blockDim.x;
    if (e < n) lds[(e / C) * RS + e % C] = pf[i];
  }
}

template <class T, int C>
__device__ __forceinline__ void axpy_row(T (&acc)[C], T coef, const T* x) {
#pragma unroll
  for (int c = 0; c < C; c++) acc[c] += coef * x[c];
}

// Rows kernel: neutron-neutron and proton-neutron parts of W for one proton row of one
// block (App. B). One lane owns one target n' and all C columns of the tile. For every
// proton jump p' -> p the source row V[p, :, tile] is staged in LDS; the lane then
// gathers through its neutron jumps n' -> n (staged per class in LDS) with the element
// h(a b c d) of the class table (the row of the proton op, staged per class in LDS).
template <class T, int C, int MAXP>
__global__ __launch_bounds__(1024) void hv_rows_kernel(HVArgs<T> a) {
  extern __shared__ __align__(16) char smem_[];
  constexpr int RS = row_stride<T, C>();
  T* row = reinterpret_cast<T*>(smem_);
  int2* ent = reinterpret_cast<int2*>(smem_ + a.row_bytes);
  T* hs = reinterpret_cast<T*>(smem_ + a.row_bytes + a.ent_bytes);
  const int entcap = (int)(a.ent_bytes / sizeof(int2));
  const int hscap = (int)(a.hs_bytes / sizeof(T));
  const int64_t nitems = a.item0[a.nblocks];
  const int64_t item = xcd_item(blockIdx.x, nitems);
  if (item >= nitems) return;
  const int b = find_block(a.item0, a.nblocks, item);
  int64_t rel = item - a.item0[b];
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
  const int thi = min(dn, tlo + nthr * MAXP);
  T acc[MAXP][C];
#pragma unroll
  for (int q = 0; q < MAXP; q++)
#pragma unroll
    for (int c = 0; c < C; c++) acc[q][c] = T(0);

  // own row: neutron-neutron part (single-particle energies included)
  stage<T, C>(row, a.V + (off + (int64_t)pl * dn) * a.ldv + c0, a.ldv, dn, cvalid);
  int st_blk = b, st_row = pl;
  __syncthreads();
  const int ns0l = a.blk_nslice0[b];
#pragma unroll
  for (int q = 0; q < MAXP; q++) {
    const int n = tlo + q * nthr + tid;
    if (n < thi) {
      const int sl = ns0l + n / 64, ln = n % 64;
      const int base = a.ne_off[sl], wd = a.ne_w[sl];
      for (int k = 0; k < wd; k++) {
        const int at = base + k * 64 + ln;
        axpy_row<T, C>(acc[q], a.ne_val[at], row + a.ne_col[at] * RS);
      }
    }
  }
  // proton-neutron part, class by class
  const int ncl = a.ncl;
  for (int cls = 0; cls < ncl; cls++) {
    const int sb = a.src_blk[b * ncl + cls];
    if (sb < 0) continue;
    const int j0 = a.pj_start[gp * ncl + cls], j1 = a.pj_start[gp * ncl + cls + 1];
    if (j0 == j1) continue;
    const int cn = (2 * a.tjmax - cls / 2) * 2 + (cls & 1);
    const int* ns0 = a.nj_start + (int64_t)cn * (a.nn_total + 1) + gn0;
    const int ebase = ns0[tlo], eend = ns0[thi];
    const bool ent_lds = (eend - ebase) <= entcap;
    const int hn = a.h_ncol[cls];
    const T* hg = a.h + a.h_off[cls];
    const bool hs_lds = (j1 - j0) * hn <= hscap;
    __syncthreads();  // previous users of ent / hs / row are done
    if (ent_lds)
      for (int e = tid; e < eend - ebase; e += nthr) ent[e] = a.nj_pack[ebase + e];
    if (hs_lds)
      for (int e = tid; e < (j1 - j0) * hn; e += nthr) {
        const int jj = e / hn, o = e % hn;
        hs[e] = hg[(a.pj_meta[j0 + jj] >> 1) * hn + o];
      }
    int kb[MAXP], ke[MAXP];
#pragma unroll
    for (int q = 0; q < MAXP; q++) {
      const int n = tlo + q * nthr + tid;
      kb[q] = (n < thi) ? ns0[n] - ebase : 0;
      ke[q] = (n < thi) ? ns0[n + 1] - ebase : 0;
    }
    const int2* E = ent_lds ? ent : (a.nj_pack + ebase);
    const int64_t soff = a.blk_off[sb];
    const int sdn = a.blk_dn[sb];
    const bool can_pf = sdn * C <= MAXPF * nthr;
    __syncthreads();
    // groups of jumps with the same source row; the next group's row is prefetched
    int jg = j0;
    while (jg < j1) {
      const int p = a.pj_idx[jg];
      int je = jg + 1;
      while (je < j1 && a.pj_idx[je] == p) je++;
      if (p != st_row || sb != st_blk) {
        __syncthreads();
        stage<T, C>(row, a.V + (soff + (int64_t)p * sdn) * a.ldv + c0, a.ldv, sdn, cvalid);
        st_blk = sb;
        st_row = p;
        __syncthreads();
      }
      T pf[MAXPF];
      const bool pfn = can_pf && je < j1;
      if (pfn) prefetch<T, C>(pf, a.V + (soff + (int64_t)a.pj_idx[je] * sdn) * a.ldv + c0, a.ldv, sdn, cvalid);
      for (int j = jg; j < je; j++) {
        const int pm = a.pj_meta[j];
        const T* hr = hs_lds ? hs + (j - j0) * hn : hg + (pm >> 1) * hn;
        const T sj = (pm & 1) ? T(-1) : T(1);
#pragma unroll
        for (int q = 0; q < MAXP; q++) {
          for (int k = kb[q]; k < ke[q]; k++) {
            const int2 e = E[k];
            const T hv = ((e.y & 1) ? -sj : sj) * hr[e.y >> 1];
            axpy_row<T, C>(acc[q], hv, row + e.x * RS);
          }
        }
      }
      if (pfn) {
        __syncthreads();
        commit<T, C>(row, pf, sdn);
        st_row = a.pj_idx[je];
        st_blk = sb;
        __syncthreads();
      }
      jg = je;
    }
  }
#pragma unroll
  for (int q = 0; q < MAXP; q++) {
    const int n = tlo + q * nthr + tid;
    if (n < thi) {
      T* w = a.W + (off + (int64_t)pl * dn + n) * a.ldw + c0;
#pragma unroll
      for (int c = 0; c < C; c++)
        if (c < cvalid) w[c] = acc[q][c];
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
  const int gp0 = a.blk_p0[b];
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

static int pow2ceil(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

static int rs_of(int C, size_t elt) { return elt == 8 ? (C >= 2 ? C + 2 : 2) : (C >= 4 ? C + 4 : 4); }

static HVPlan& plan_for(const Model& m, int nb, size_t elt) {
  const int key = nb * 16 + (int)elt;
  auto it = m.hv_plans.find(key);
  if (it != m.hv_plans.end()) return *it->second;
  auto owned = std::make_unique<HVPlan>();
  HVPlan* P = owned.get();
  const size_t lds_max = 160 * 1024, row_budget = 100 * 1024;
  const int maxrows = std::max(m.max_dn, m.max_dp);
  int C = std::min(32, pow2ceil(nb));
  while (C > 1 && (size_t)maxrows * rs_of(C, elt) * elt > row_budget) C >>= 1;
  TRBL_REQUIRE((size_t)maxrows * rs_of(C, elt) * elt <= lds_max - 16 * 1024, TRBL_E_INVALID,
               "sector too large for the LDS tile");
  P->C = C;
  P->ntile = (nb + C - 1) / C;
  // threads: one lane per target; up to 4 targets per lane, then chunks
  auto pick = [&](int d, int& nthr, int& maxp, int& nchunk) {
    nthr = std::min(1024, std::max(64, (d + 63) / 64 * 64));
    maxp = 1;
    while (maxp < 4 && nthr * maxp < d) maxp <<= 1;
    nchunk = (d + nthr * maxp - 1) / (nthr * maxp);
  };
  pick(m.max_dn, P->nthr_r, P->maxp_r, P->nchunk_r);
  pick(m.max_dp, P->nthr_c, P->maxp_c, P->nchunk_c);
  std::vector<int64_t> i0(m.blocks.size() + 1, 0), c0(m.blocks.size() + 1, 0);
  for (size_t b = 0; b < m.blocks.size(); b++) {
    i0[b + 1] = i0[b] + (int64_t)m.blocks[b].dp * P->ntile * P->nchunk_r;
    c0[b + 1] = c0[b] + (int64_t)m.blocks[b].dn * P->ntile * P->nchunk_c;
  }
  P->rows_items = i0.back();
  P->cols_items = c0.back();
  P->item0.upload(i0);
  P->citem0.upload(c0);
  P->row_bytes = ((size_t)m.max_dn * rs_of(C, elt) * elt + 15) / 16 * 16;
  const size_t rest = lds_max - P->row_bytes;
  P->hs_bytes = std::min<size_t>(16 * 1024, rest / 4) / 16 * 16;
  P->ent_bytes = std::min<size_t>(64 * 1024, rest - P->hs_bytes) / 16 * 16;
  P->shm_r = P->row_bytes + P->ent_bytes + P->hs_bytes;
  P->shm_c = ((size_t)m.max_dp * rs_of(C, elt) * elt + 15) / 16 * 16;
  m.hv_plans[key] = std::move(owned);
  return *P;
}

template <class T>
static HVArgs<T> make_args(const Model& m, int nb, const void* V, int64_t ldv, void* W, int64_t ldw) {
  HVArgs<T> a;
  a.V = static_cast<const T*>(V);
  a.W = static_cast<T*>(W);
  a.ldv = ldv;
  a.ldw = ldw;
  a.nb = nb;
  a.nblocks = (int)m.blocks.size();
  a.ncl = m.cl.nclass;
  a.tjmax = m.cl.tjmax;
  a.nn_total = m.nn_total;
  const DeviceTables& d = m.dt;
  a.blk_dp = d.blk_dp.as<int>();
  a.blk_dn = d.blk_dn.as<int>();
  a.blk_off = d.blk_off.as<int64_t>();
  a.blk_p0 = d.blk_p0.as<int>();
  a.blk_n0 = d.blk_n0.as<int>();
  a.src_blk = d.src_blk.as<int>();
  a.pj_start = d.pj_start.as<int>();
  a.pj_idx = d.pj_idx.as<int>();
  a.pj_meta = d.pj_meta.as<int>();
  a.nj_start = d.nj_start.as<int>();
  a.nj_pack = d.nj_pack.as<int2>();
  a.h_off = d.h_off.as<int>();
  a.h_ncol = d.h_ncol.as<int>();
  a.pp_ptr = d.pp_ptr.as<int>();
  a.pp_col = d.pp_col.as<int>();
  a.nn_ptr = d.nn_ptr.as<int>();
  a.nn_col = d.nn_col.as<int>();
  a.pe_off = d.pe_off.as<int>();
  a.pe_w = d.pe_w.as<int>();
  a.pe_col = d.pe_col.as<int>();
  a.ne_off = d.ne_off.as<int>();
  a.ne_w = d.ne_w.as<int>();
  a.ne_col = d.ne_col.as<int>();
  a.blk_pslice0 = d.blk_pslice0.as<int>();
  a.blk_nslice0 = d.blk_nslice0.as<int>();
  if constexpr (sizeof(T) == 8) {
    a.pe_val = d.pe_v64.as<T>();
    a.ne_val = d.ne_v64.as<T>();
    a.h = d.h64.as<T>();
    a.pp_val = d.pp_v64.as<T>();
    a.nn_val = d.nn_v64.as<T>();
  } else {
    a.pe_val = d.pe_v32.as<T>();
    a.ne_val = d.ne_v32.as<T>();
    a.h = d.h32.as<T>();
    a.pp_val = d.pp_v32.as<T>();
    a.nn_val = d.nn_v32.as<T>();
  }
  return a;
}

template <class T, int C, int MP>
static void launch_rows(const HVArgs<T>& a, const HVPlan& P, hipStream_t s) {
  hipLaunchKernelGGL((hv_rows_kernel<T, C, MP>), dim3((unsigned)((P.rows_items + 7) / 8 * 8)), dim3(P.nthr_r),
                     P.shm_r, s, a);
}
template <class T, int C, int MP>
static void launch_cols(const HVArgs<T>& a, const HVPlan& P, hipStream_t s) {
  hipLaunchKernelGGL((hv_cols_kernel<T, C, MP>), dim3((unsigned)((P.cols_items + 7) / 8 * 8)), dim3(P.nthr_c),
                     P.shm_c, s, a);
}

template <class T, int C>
static void dispatch_c(HVArgs<T>& a, const HVPlan& P, hipStream_t s) {
  a.nchunk = P.nchunk_r;
  if (P.maxp_r == 1) launch_rows<T, C, 1>(a, P, s);
  else if (P.maxp_r == 2) launch_rows<T, C, 2>(a, P, s);
  else launch_rows<T, C, 4>(a, P, s);
  a.nchunk = P.nchunk_c;
  if (P.maxp_c == 1) launch_cols<T, C, 1>(a, P, s);
  else if (P.maxp_c == 2) launch_cols<T, C, 2>(a, P, s);
  else launch_cols<T, C, 4>(a, P, s);
}

template <class T>
static void run_hv(const Model& m, int nb, const void* V, int64_t ldv, void* W, int64_t ldw, hipStream_t s) {
  HVPlan& P = plan_for(m, nb, sizeof(T));
  HVArgs<T> a = make_args<T>(m, nb, V, ldv, W, ldw);
  a.C = P.C;
  a.ntile = P.ntile;
  a.item0 = P.item0.as<int64_t>();
  a.citem0 = P.citem0.as<int64_t>();
  a.row_bytes = P.row_bytes;
  a.ent_bytes = P.ent_bytes;
  a.hs_bytes = P.hs_bytes;
  TRBL_REQUIRE(P.rows_items < (int64_t)1 << 31 && P.cols_items < (int64_t)1 << 31, TRBL_E_INVALID,
               "problem too large for one launch");
  switch (P.C) {
    case 1: dispatch_c<T, 1>(a, P, s); break;
    case 2: dispatch_c<T, 2>(a, P, s); break;
    case 4: dispatch_c<T, 4>(a, P, s); break;
    case 8: dispatch_c<T, 8>(a, P, s); break;
    case 16: dispatch_c<T, 16>(a, P, s); break;
    default: dispatch_c<T, 32>(a, P, s); break;
  }
}

void launch_apply(const Model& m, int precision, int nb, const void* V, int64_t ldv, void* W, int64_t ldw,
                  hipStream_t s) {
  TRBL_REQUIRE(m.has_h, TRBL_E_STATE, "no Hamiltonian set");
  TRBL_REQUIRE(nb >= 1 && nb <= 64, TRBL_E_INVALID, "nb must be 1..64");
  TRBL_REQUIRE(ldv >= nb && ldw >= nb, TRBL_E_INVALID, "leading dimension smaller than nb");
  TRBL_REQUIRE(V && W && V != W, TRBL_E_INVALID, "V and W must be distinct device buffers");
  if (precision == TRBL_FP64) run_hv<double>(m, nb, V, ldv, W, ldw, s);
  else run_hv<float>(m, nb, V, ldv, W, ldw, s);
  TRBL_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ basis indexing on the device
struct RankArgs {
  int ns, norb;
  int tm[64];
  int orb[64];
  int lpar[64];                  // l parity of each state's orbit
  int nsec[2];
  const int* sec_start[2];
  const int* sec_size[2];
  const int* sec_twoM[2];
  const int* sec_par[2];
  const uint64_t* words[2];
  const uint64_t* part[2];
  const int* blk_of_sec;
  int nnsec;
  const int64_t* blk_off;
  const int* blk_dn;
  int nblocks;
  const int* blk_p0;
  const int* blk_n0;
};

__device__ static uint64_t rev_bits(uint64_t w, int ns) { return __brevll(w) >> (64 - ns); }

// rank of word w inside its species sector, or -1
__device__ static int species_rank(const RankArgs& a, int s, uint64_t w, int* sector) {
  *sector = -1;
  if (a.ns < 64 && (w >> a.ns)) return -1;
  int tm = 0, lp = 0;
  int cnt[12] = {0};
  for (uint64_t x = w; x; x &= x - 1) {
    const int q = __ffsll((long long)x) - 1;
    tm += a.tm[q];
    lp += a.lpar[q];
    cnt[a.orb[q]]++;
  }
  const int par = (lp & 1) ? -1 : 1;
  int k = -1;
  for (int i = 0; i < a.nsec[s]; i++)
    if (a.sec_twoM[s][i] == tm && a.sec_par[s][i] == par) {
      k = i;
      break;
    }
  *sector = k;
  if (k < 0) return -1;
  uint64_t pk = 0;
  for (int o = 0; o < a.norb; o++) pk = (pk << 5) | (uint64_t)cnt[o];
  const uint64_t rv = rev_bits(w, a.ns);
  // sector order: partition key descending, then reversed word descending
  int lo = 0, hi = a.sec_size[s][k] - 1;
  const int st = a.sec_start[s][k];
  while (lo <= hi) {
    const int mid = (lo + hi) >> 1;
    const uint64_t mp = a.part[s][st + mid];
    const uint64_t mr = rev_bits(a.words[s][st + mid], a.ns);
    if (mp == pk && mr == rv) return mid;
    const bool before = (mp > pk) || (mp == pk && mr > rv);  // element sorts before the key
    if (before) lo = mid + 1;
    else hi = mid - 1;
  }
  return -1;
}

__global__ void rank_kernel(RankArgs a, const uint64_t* pb, const uint64_t* nbits, int64_t n, int64_t* out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  int kp, kn;
  const int rp = species_rank(a, 0, pb[i], &kp);
  const int rn = species_rank(a, 1, nbits[i], &kn);
  int64_t r = -1;
  if (rp >= 0 && rn >= 0) {
    const int b = a.blk_of_sec[kp * a.nnsec + kn];
    if (b >= 0) r = a.blk_off[b] + (int64_t)rp * a.blk_dn[b] + rn;
  }
  out[i] = r;
}

__global__ void unrank_kernel(RankArgs a, const int64_t* idx, int64_t n, uint64_t* pb, uint64_t* nbits) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t x = idx[i];
  if (x < 0 || x >= a.blk_off[a.nblocks]) {
    pb[i] = ~0ull;
    nbits[i] = ~0ull;
    return;
  }
  int lo = 0, hi = a.nblocks - 1;
  while (lo < hi) {  // last block with offset <= x
    const int mid = (lo + hi + 1) >> 1;
    if (a.blk_off[mid] <= x) lo = mid;
    else hi = mid - 1;
  }
  const int64_t rel = x - a.blk_off[lo];
  const int dn = a.blk_dn[lo];
  pb[i] = a.words[0][a.blk_p0[lo] + rel / dn];
  nbits[i] = a.words[1][a.blk_n0[lo] + rel % dn];
}

static RankArgs rank_args(const Model& m) {
  RankArgs a{};
  a.ns = m.ns;
  a.norb = (int)m.orbits.size();
  for (int s = 0; s < m.ns; s++) {
    a.tm[s] = m.st_tm[s];
    a.orb[s] = m.st_orb[s];
    a.lpar[s] = m.orbits[m.st_orb[s]].l & 1;
  }
  for (int s = 0; s < 2; s++) {
    a.sec_twoM[s] = (s == 0 ? m.dt.psec_tm : m.dt.nsec_tm).as<int>();
    a.sec_par[s] = (s == 0 ? m.dt.psec_par : m.dt.nsec_par).as<int>();
    a.nsec[s] = (int)m.sp[s].sectors.size();
    a.sec_start[s] = (s == 0 ? m.dt.psec_start : m.dt.nsec_start).as<int>();
    a.sec_size[s] = (s == 0 ? m.dt.psec_size : m.dt.nsec_size).as<int>();
    a.words[s] = (s == 0 ? m.dt.pwords : m.dt.nwords).as<uint64_t>();
    a.part[s] = (s == 0 ? m.dt.ppart : m.dt.npart).as<uint64_t>();
  }
  a.blk_of_sec = m.dt.blk_of_sec.as<int>();
  a.nnsec = (int)m.sp[1].sectors.size();
  a.blk_off = m.dt.blk_off.as<int64_t>();
  a.blk_dn = m.dt.blk_dn.as<int>();
  a.nblocks = (int)m.blocks.size();
  a.blk_p0 = m.dt.blk_p0.as<int>();
  a.blk_n0 = m.dt.blk_n0.as<int>();
  return a;
}

void launch_rank(const Model& m, const uint64_t* pb, const uint64_t* nbits, int64_t n, int64_t* idx, hipStream_t s) {
  if (n <= 0) return;
  RankArgs a = rank_args(m);
  const int64_t nbk = (n + 255) / 256;
  hipLaunchKernelGGL(rank_kernel, dim3((unsigned)nbk), dim3(256), 0, s, a, pb, nbits, n, idx);
  TRBL_HIP(hipGetLastError());
}

void launch_unrank(const Model& m, const int64_t* idx, int64_t n, uint64_t* pb, uint64_t* nbits, hipStream_t s) {
  if (n <= 0) return;
  RankArgs a = rank_args(m);
  const int64_t nbk = (n + 255) / 256;
  hipLaunchKernelGGL(unrank_kernel, dim3((unsigned)nbk), dim3(256), 0, s, a, idx, n, pb, nbits);
  TRBL_HIP(hipGetLastError());
}

}  // namespace trbl
