// Block H.V for spaces of one species (the other species empty), with the identical-particle
// part of App. B generated per element instead of being stored: the single-species workloads
// of Sec. 4.2 have sectors of millions of determinants, far beyond what the LDS-staged rows
// kernel can hold and too many elements to tabulate. Sources are ranked with a two-level
// table (App. A: a determinant's position from its bit string).
//
// Two-level ranking. The m-states are split into a low part of `half` states and a high
// part. The determinants of one sector (N, 2M, parity) with low pattern l are exactly the
// high patterns r of the class (N - |l|, 2M - 2M(l), parity * parity(l)), so
//   internal(w) = base[sector][l] + rank[r]
// numbers a sector densely (rank: position of r among the high patterns of its class in
// increasing order; base: running sum over the low patterns of the size of their class).
// perm maps the internal number to the Table-1 position inside the sector. The product runs
// in the internal order: V is gathered into it once, the kernel reads sources at their
// internal numbers (determinants that differ only in the high part stay inside one low
// pattern's contiguous range, which keeps many sources of neighbouring targets together),
// and W is scattered back to Table-1 order.
#include <map>
#include <tuple>

#include "internal.h"

namespace trbl {

void build_fly_basis(Model& m) {
  const Species& S = m.sp[m.fly_s];
  const int ns = m.ns;
  TRBL_REQUIRE(ns <= 44, TRBL_E_TOO_MANY, "single-species spaces of more than 44 m-states are not supported");
  const int half = ns / 2, high = ns - half;
  m.fly_half = half;
  auto key_of = [&](uint64_t x, int shift) {  // (count, 2M, odd parity) of a pattern of states
    int n = 0, tm = 0, lsum = 0;
    for (uint64_t y = x; y; y &= y - 1) {
      const int s = __builtin_ctzll(y) + shift;
      n++;
      tm += m.st_tm[s];
      lsum += m.orbits[m.st_orb[s]].l;
    }
    return std::make_tuple(n, tm, lsum & 1);
  };
  std::map<std::tuple<int, int, int>, int> count;
  std::vector<int> rank((size_t)1 << high);
  for (uint64_t r = 0; r < (1ull << high); r++) rank[r] = count[key_of(r, half)]++;
  const int nsec = (int)S.sectors.size();
  std::vector<int> base((size_t)nsec << half), perm(S.words.size()), sstart(nsec);
  std::vector<uint64_t> wint(S.words.size());
  std::vector<int64_t> soff(nsec + 1, -1);
  for (int k = 0; k < nsec; k++) {
    const SpeciesSector& q = S.sectors[k];
    int run = 0;
    for (uint64_t l = 0; l < (1ull << half); l++) {
      base[((size_t)k << half) | l] = run;
      const auto lk = key_of(l, 0);
      const int need = S.npart - std::get<0>(lk);
      if (need < 0) continue;
      const auto it = count.find({need, q.twoM - std::get<1>(lk), (q.par < 0 ? 1 : 0) ^ std::get<2>(lk)});
      if (it != count.end()) run += it->second;
    }
    TRBL_REQUIRE(run == q.size, TRBL_E_INVALID, "two-level ranking does not reproduce the sector");
    for (int i = 0; i < q.size; i++) {
      const uint64_t w = S.words[q.start + i];
      const int in = base[((size_t)k << half) | (w & ((1ull << half) - 1))] + rank[w >> half];
      perm[q.start + in] = i;
      wint[q.start + in] = w;
    }
    sstart[k] = q.start;
    for (const auto& b : m.blocks)
      if ((m.fly_s == 1 ? b.nsec : b.psec) == k) soff[k] = b.off;
    TRBL_REQUIRE(soff[k] >= 0, TRBL_E_INVALID, "sector without a block");
  }
  soff[nsec] = m.dim;
  m.dt.fly_base.upload(base);
  m.dt.fly_rank.upload(rank);
  m.dt.fly_perm.upload(perm);
  m.dt.fly_wint.upload(wint);
  m.dt.fly_soff.upload(soff);
  m.dt.fly_sstart.upload(sstart);
}

// two-body terms of the occupied species grouped by creation pair (a < b), and the
// single-particle energy of every m-state
void build_fly_terms(Model& m) {
  const int ns = m.ns;
  const std::vector<MTerm>& T = m.fly_s == 1 ? m.terms_nn : m.terms_pp;
  std::vector<std::vector<int>> by_pair((size_t)ns * ns);
  for (int k = 0; k < (int)T.size(); k++) by_pair[(size_t)T[k].a * ns + T[k].b].push_back(k);
  std::vector<int> pstart(1, 0), cd;
  std::vector<double> h;
  for (const auto& lst : by_pair) {
    for (int k : lst) {
      cd.push_back(T[k].c);
      cd.push_back(T[k].d);
      h.push_back(T[k].h);
    }
    pstart.push_back((int)h.size());
  }
  std::vector<double> e(ns);
  for (int s = 0; s < ns; s++) e[s] = m.spe[m.fly_s][m.st_orb[s]];
  m.dt.fly_pstart.upload(pstart);
  if (cd.empty()) cd.assign(2, 0);
  if (h.empty()) h.assign(1, 0.0);
  m.dt.fly_cd.upload(cd);
  m.dt.fly_h64.upload(h);
  m.dt.fly_h32.upload(std::vector<float>(h.begin(), h.end()));
  m.dt.fly_e64.upload(e);
  m.dt.fly_e32.upload(std::vector<float>(e.begin(), e.end()));
}

template <class T>
struct FlyArgs {
  const T* V;
  T* W;
  int64_t ldv, ldw, D;
  int nb, ns, half, nsec;
  const int* sstart;     // first species index of each sector (internal numbering starts there too)
  const uint64_t* words;  // determinants in the internal order
  const int* base;
  const int* rank;
  const int* pstart;
  const int2* cd;
  const T* h;
  const T* e;
  const double* mask;    // optional, Table-1 order: targets with mask 0 get W = 0 without work
  const int* perm;       // internal -> Table-1 position inside the sector (with mask)
  const int64_t* soff;   // first M-scheme index of each sector (with mask)
};

__device__ __forceinline__ int jw_odd(uint64_t w, int s) { return __popcll(w & ((1ull << s) - 1)) & 1; }

// One thread per target determinant w (internal order) and C columns: W[w] = (sum of the
// single-particle energies of w) V[w] + sum over occupied pairs a < b and terms (c, d) of that
// creation pair of sign * h * V[source], source = w with a, b removed and d, c added (the
// adjoint of the term c+_a c+_b c_d c_c applied to w), the sign counting the occupied states
// below each operator. V and W are in the internal order, nb columns apart.
template <class T, int C>
__global__ __launch_bounds__(256) void fly_kernel(FlyArgs<T> a) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= a.D) return;
  const int c0 = blockIdx.y * C, cv = min(C, a.nb - c0);
  int k = 0;
  while (k + 1 < a.nsec && t >= a.sstart[k + 1]) k++;
  const int64_t st = a.sstart[k];
  const int* bk = a.base + ((int64_t)k << a.half);
  const uint64_t w = a.words[t];
  const uint64_t lmask = (1ull << a.half) - 1;
  if (a.mask && a.mask[a.soff[k] + a.perm[t]] == 0.0) {  // outside a truncated space
    T* wt = a.W + t * a.nb + c0;
    for (int c = 0; c < cv; c++) wt[c] = T(0);
    return;
  }
  T acc[C];
  T e = T(0);
  for (uint64_t x = w; x; x &= x - 1) e += a.e[__builtin_ctzll(x)];
  const T* vt = a.V + t * a.nb + c0;
#pragma unroll
  for (int c = 0; c < C; c++) acc[c] = c < cv ? e * vt[c] : T(0);
  for (uint64_t x = w; x; x &= x - 1) {
    const int sa = __builtin_ctzll(x);
    for (uint64_t y = x & (x - 1); y; y &= y - 1) {
      const int sb = __builtin_ctzll(y);
      const int q0 = a.pstart[sa * a.ns + sb], q1 = a.pstart[sa * a.ns + sb + 1];
      if (q0 == q1) continue;
      uint64_t r0 = w;
      int sg = jw_odd(r0, sa);
      r0 &= ~(1ull << sa);
      sg ^= jw_odd(r0, sb);
      r0 &= ~(1ull << sb);
      for (int q = q0; q < q1; q++) {
        const int2 p = a.cd[q];  // (c, d)
        uint64_t r = r0;
        if ((r >> p.y) & 1) continue;
        int s2 = sg ^ jw_odd(r, p.y);
        r |= 1ull << p.y;
        if ((r >> p.x) & 1) continue;
        s2 ^= jw_odd(r, p.x);
        r |= 1ull << p.x;
        const int64_t j = st + bk[r & lmask] + a.rank[r >> a.half];
        const T hv = s2 ? -a.h[q] : a.h[q];
        const T* vs = a.V + j * a.nb + c0;
#pragma unroll
        for (int c = 0; c < C; c++)
          if (c < cv) acc[c] += hv * vs[c];
      }
    }
  }
  T* wt = a.W + t * a.nb + c0;
#pragma unroll
  for (int c = 0; c < C; c++)
    if (c < cv) wt[c] = acc[c];
}

// rows between the Table-1 order (leading dimension ld) and the internal order (packed, nb):
// internal row i of sector k is Table-1 row soff[k] + perm[i]
template <class T>
__global__ void fly_permute_kernel(const T* src, int64_t lds_, T* dst, int64_t ldd, int nb, int64_t n, int nsec,
                                   const int* sstart, const int64_t* soff, const int* perm, int to_internal) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n * nb; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / nb;
    const int c = (int)(e - i * nb);
    int k = 0;
    while (k + 1 < nsec && i >= sstart[k + 1]) k++;
    const int64_t row = soff[k] + perm[i];
    if (to_internal) dst[i * ldd + c] = src[row * lds_ + c];
    else dst[row * ldd + c] = src[i * lds_ + c];
  }
}

template <class T>
static void run_fly(const Model& m, int nb, const void* V, int64_t ldv, void* W, int64_t ldw, const double* mask,
                    hipStream_t s) {
  FlyArgs<T> a{};
  const int64_t D = m.dim;
  const DeviceTables& d = m.dt;
  // internal-order copies of V and W, kept with the model for the next product
  DevBuf& buf = m.fly_buf[sizeof(T) == 8 ? 1 : 0];
  buf.alloc((size_t)2 * D * nb * sizeof(T));
  T* vin = buf.as<T>();
  T* win = vin + D * nb;
  const int nsec = (int)m.sp[m.fly_s].sectors.size();
  const int64_t ne = D * nb;
  const unsigned g1 = elementwise_grid(ne);
  hipLaunchKernelGGL((fly_permute_kernel<T>), dim3(g1), dim3(256), 0, s, static_cast<const T*>(V), ldv, vin,
                     (int64_t)nb, nb, D, nsec, d.fly_sstart.as<int>(), d.fly_soff.as<int64_t>(),
                     d.fly_perm.as<int>(), 1);
  a.V = vin;
  a.W = win;
  a.D = D;
  a.nb = nb;
  a.ns = m.ns;
  a.half = m.fly_half;
  a.nsec = nsec;
  a.sstart = d.fly_sstart.as<int>();
  a.words = d.fly_wint.as<uint64_t>();
  a.base = d.fly_base.as<int>();
  a.rank = d.fly_rank.as<int>();
  a.pstart = d.fly_pstart.as<int>();
  a.cd = d.fly_cd.as<int2>();
  a.mask = mask;
  a.perm = d.fly_perm.as<int>();
  a.soff = d.fly_soff.as<int64_t>();
  if constexpr (sizeof(T) == 8) {
    a.h = d.fly_h64.as<T>();
    a.e = d.fly_e64.as<T>();
  } else {
    a.h = d.fly_h32.as<T>();
    a.e = d.fly_e32.as<T>();
  }
  // the two-body part by pair blocks (the diagonal in its final pass); products restricted to a
  // truncated space keep the per-element kernel, which does not generate the rows outside it
  if (m.flyt.on && !mask) {
    launch_fly_tiles<T>(m, nb, vin, win, mask, s);
  } else if (nb <= 8) {
    const dim3 grid((unsigned)((D + 255) / 256), 1);
    hipLaunchKernelGGL((fly_kernel<T, 8>), grid, dim3(256), 0, s, a);
  } else {
    const dim3 grid((unsigned)((D + 255) / 256), (unsigned)((nb + 15) / 16));
    hipLaunchKernelGGL((fly_kernel<T, 16>), grid, dim3(256), 0, s, a);
  }
  hipLaunchKernelGGL((fly_permute_kernel<T>), dim3(g1), dim3(256), 0, s, win, (int64_t)nb, static_cast<T*>(W), ldw,
                     nb, D, nsec, d.fly_sstart.as<int>(), d.fly_soff.as<int64_t>(), d.fly_perm.as<int>(), 0);
}

void launch_fly(const Model& m, int precision, int nb, const void* V, int64_t ldv, void* W, int64_t ldw,
                hipStream_t s, const double* mask) {
  if (precision == TRBL_FP64) run_fly<double>(m, nb, V, ldv, W, ldw, mask, s);
  else run_fly<float>(m, nb, V, ldv, W, ldw, mask, s);
  TRBL_HIP(hipGetLastError());
}

}  // namespace trbl
