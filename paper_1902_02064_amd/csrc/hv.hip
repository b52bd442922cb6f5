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
  int nb, tpt;  // vectors, targets per workgroup chunk
  int nblocks, ncl, tjmax;
  const int* blk_dp;
  const int* blk_dn;
  const int64_t* blk_off;
  const int* blk_p0;
  const int* blk_n0;
  const int* src_blk;
  const int* pj_start;
  const int* pj_idx;
  const int* pj_meta;
  const int* nj_start;
  const int* nj_idx;
  const int* nj_meta;
  const int* h_off;
  const int* h_ncol;
  const T* h;
  const int* pp_ptr;
  const int* pp_col;
  const T* pp_val;
  const int* nn_ptr;
  const int* nn_col;
  const T* nn_val;
};

template <class T>
__global__ __launch_bounds__(256) void hv_rows_kernel(HVArgs<T> a) {
  // locate (block, proton row, chunk of neutron targets) of this workgroup
  const int64_t item = blockIdx.x;
  int b = 0, chunks = 1;
  int64_t base = 0;
  for (; b < a.nblocks; b++) {
    chunks = (a.blk_dn[b] + a.tpt - 1) / a.tpt;
    const int64_t cnt = (int64_t)a.blk_dp[b] * chunks;
    if (item < base + cnt) break;
    base += cnt;
  }
  if (b >= a.nblocks) return;
  const int64_t rel = item - base;
  const int pl = (int)(rel / chunks);
  const int ch = (int)(rel % chunks);
  const int tid = threadIdx.x;
  const int c = tid % a.nb;
  const int slot = tid / a.nb;
  const int dn = a.blk_dn[b];
  const int nt = ch * a.tpt + slot;
  if (slot >= a.tpt || nt >= dn) return;
  const int64_t off = a.blk_off[b];
  const int gp = a.blk_p0[b] + pl;
  const int gn = a.blk_n0[b] + nt;
  const int ncl = a.ncl;
  T acc = 0;
  // identical-particle operators (include single-particle energies on the diagonal)
  for (int e = a.pp_ptr[gp]; e < a.pp_ptr[gp + 1]; e++)
    acc += a.pp_val[e] * a.V[(off + (int64_t)a.pp_col[e] * dn + nt) * a.ldv + c];
  for (int e = a.nn_ptr[gn]; e < a.nn_ptr[gn + 1]; e++)
    acc += a.nn_val[e] * a.V[(off + (int64_t)pl * dn + a.nn_col[e]) * a.ldv + c];
  // proton-neutron part through one-body jumps
  for (int cls = 0; cls < ncl; cls++) {
    const int sb = a.src_blk[b * ncl + cls];
    if (sb < 0) continue;
    const int j0 = a.pj_start[gp * ncl + cls], j1 = a.pj_start[gp * ncl + cls + 1];
    if (j0 == j1) continue;
    const int cn = (2 * a.tjmax - cls / 2) * 2 + (cls & 1);
    const int k0 = a.nj_start[gn * ncl + cn], k1 = a.nj_start[gn * ncl + cn + 1];
    if (k0 == k1) continue;
    const int64_t soff = a.blk_off[sb];
    const int sdn = a.blk_dn[sb];
    const T* h0 = a.h + a.h_off[cls];
    const int hn = a.h_ncol[cls];
    for (int j = j0; j < j1; j++) {
      const int pm = a.pj_meta[j];
      const T* hr = h0 + (pm >> 1) * hn;
      const T* src = a.V + (soff + (int64_t)a.pj_idx[j] * sdn) * a.ldv + c;
      T part = 0;
      for (int k = k0; k < k1; k++) {
        const int nm = a.nj_meta[k];
        const T x = src[(int64_t)a.nj_idx[k] * a.ldv];
        const T hv = hr[nm >> 1];
        part += (nm & 1) ? -hv * x : hv * x;
      }
      acc += (pm & 1) ? -part : part;
    }
  }
  a.W[(off + (int64_t)pl * dn + nt) * a.ldw + c] = acc;
}

template <class T>
static HVArgs<T> make_args(const Model& m, int nb, const void* V, int64_t ldv, void* W, int64_t ldw) {
  HVArgs<T> a;
  a.V = static_cast<const T*>(V);
  a.W = static_cast<T*>(W);
  a.ldv = ldv;
  a.ldw = ldw;
  a.nb = nb;
  a.tpt = 256 / nb;
  a.nblocks = (int)m.blocks.size();
  a.ncl = m.cl.nclass;
  a.tjmax = m.cl.tjmax;
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
  a.nj_idx = d.nj_idx.as<int>();
  a.nj_meta = d.nj_meta.as<int>();
  a.h_off = d.h_off.as<int>();
  a.h_ncol = d.h_ncol.as<int>();
  a.pp_ptr = d.pp_ptr.as<int>();
  a.pp_col = d.pp_col.as<int>();
  a.nn_ptr = d.nn_ptr.as<int>();
  a.nn_col = d.nn_col.as<int>();
  if constexpr (sizeof(T) == 8) {
    a.h = d.h64.as<T>();
    a.pp_val = d.pp_v64.as<T>();
    a.nn_val = d.nn_v64.as<T>();
  } else {
    a.h = d.h32.as<T>();
    a.pp_val = d.pp_v32.as<T>();
    a.nn_val = d.nn_v32.as<T>();
  }
  return a;
}

void launch_apply(const Model& m, int precision, int nb, const void* V, int64_t ldv, void* W, int64_t ldw,
                  hipStream_t s) {
  TRBL_REQUIRE(m.has_h, TRBL_E_STATE, "no Hamiltonian set");
  TRBL_REQUIRE(nb >= 1 && nb <= 64, TRBL_E_INVALID, "nb must be 1..64");
  TRBL_REQUIRE(ldv >= nb && ldw >= nb, TRBL_E_INVALID, "leading dimension smaller than nb");
  TRBL_REQUIRE(V && W && V != W, TRBL_E_INVALID, "V and W must be distinct device buffers");
  const int tpt = 256 / nb;
  int64_t items = 0;
  for (const auto& b : m.blocks) items += (int64_t)b.dp * ((b.dn + tpt - 1) / tpt);
  TRBL_REQUIRE(items < (int64_t)1 << 31, TRBL_E_INVALID, "problem too large for one launch");
  if (precision == TRBL_FP64) {
    auto a = make_args<double>(m, nb, V, ldv, W, ldw);
    hipLaunchKernelGGL(hv_rows_kernel<double>, dim3((unsigned)items), dim3(256), 0, s, a);
  } else {
    auto a = make_args<float>(m, nb, V, ldv, W, ldw);
    hipLaunchKernelGGL(hv_rows_kernel<float>, dim3((unsigned)items), dim3(256), 0, s, a);
  }
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
