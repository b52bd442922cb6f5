// Identical-particle (two-body) part of the block H.V of single-species spaces as dense pair
// blocks on the matrix cores (App. B, the terms regrouped by their spectator nucleons).
#include <algorithm>
#include <cstdlib>
#include <map>

#include "tilecore.h"

namespace trbl {

using namespace tiles;

namespace {

// ------------------------------------------------------------------ one species: pairs of identical nucleons
// A two-body term c+_a c+_b c_d c_c (a < b, c < d) of one species leaves n - 2 nucleons in place,
// a core L. With the pairs (a, b) of one (2M, parity) listed once, the terms acting on the
// states L + a + b form the dense symmetric block h(ab; cd) restricted to pairs outside L. The
// sign of the term on L + c + d is sigma(L, a) sigma(L, b) sigma(L, c) sigma(L, d) (the operators
// act on L in the order c, d, then b, a, and a < b, c < d), a target and a source factor. Every
// term application belongs to exactly one core (the target minus a and b), so the two-body part
// of W is the sum over the C(n, 2) cores of a target, slot (position of a, position of b) each.
template <class T>
struct FlyTileArgs {
  const T* V;  // internal order, packed nb
  T* Z;
  int c0, cval, zw;  // column tile: first column, valid columns, slot row width
  int ns, half, D, vrow;
  const uint64_t* cw;  // cores, grouped
  const int* base;     // two-level ranking (sector-major low-part offsets, high-part ranks)
  const int* rank;
  const int* sstart;   // first internal index of each sector
  const int* pr_off;
  const int* pr_ab;
  const int* hb_off;
  const T* hb;
  const int* rect;    // per rectangle: pair block, target sector
  const int4* items;  // per work item: rectangle, first core, count, -
  int nitems;
};

template <class T, int DTM>
__device__ __forceinline__ void fly_store(const unsigned* Rt, const int* Pi, int d, int DT, int c, int kq, bool cok,
                                          T* Z, int64_t D, int zw, const typename Mfma<T>::acc (&acc)[DTM]) {
#pragma unroll
  for (int mt = 0; mt < DTM; mt++) {
    if (mt < DT) {
#pragma unroll
      for (int v = 0; v < 4; v++) {
        const int i = 16 * mt + Mfma<T>::row(kq, v);
        const unsigned t = Rt[i];
        const int p = Pi[i];
        if (i < d && cok)
          __builtin_nontemporal_store(flip_if((T)acc[mt][v], (unsigned)(p >> 8) & 1u),
                                      Z + ((int64_t)(p >> 9) * D + t) * zw + c);
      }
    }
  }
}

template <class T, int DTM>
__device__ __forceinline__ void fly_product(const T* Hs, const unsigned* Rv, const unsigned* Rt, const int* Pi, int d,
                                            int HW, int c, int kq, bool cok, unsigned cb, const char* Vb, T* Z,
                                            int64_t D, int zw) {
  const int KS = (d + 3) >> 2, DT = (d + 15) >> 4;
  int tb[DTM];
  typename Mfma<T>::acc acc[DTM];
#pragma unroll
  for (int mt = 0; mt < DTM; mt++) {
    tb[mt] = (Pi[16 * mt + c] & 255) * HW;
    acc[mt] = typename Mfma<T>::acc{0, 0, 0, 0};
  }
#pragma unroll
  for (int h = 0; h < DTM / 2; h++) {
    T bop[8];
    tile_loads<T>(Rv, h, kq, cb, Vb, bop);
#pragma unroll
    for (int j = 0; j < 8; j++) {
      if (8 * h + j < KS) {
        const int kk = 4 * (8 * h + j) + kq;
        const T b = flip_if(bop[j], Rv[kk] & 1u);
        const int pk = Pi[kk] & 255;
        T av[DTM];
#pragma unroll
        for (int mt = 0; mt < DTM; mt++) av[mt] = Hs[tb[mt] + pk];
#pragma unroll
        for (int mt = 0; mt < DTM; mt++)
          if (mt < DT) acc[mt] = Mfma<T>::run(av[mt], b, acc[mt]);
      }
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  fly_store<T, DTM>(Rt, Pi, d, DT, c, kq, cok, Z, D, zw, acc);
}

// Four cores of at most 16 allowed pairs each (one row tile, four steps): the 16 source loads of
// the four are issued together, then the products and stores core by core.
template <class T>
__device__ __forceinline__ void fly_batch4(const T* Hs, const unsigned (*Rv)[64], const unsigned (*Rt)[64],
                                           const int (*Pi)[64], const int (&d)[4], int HW, int c, int kq, bool cok,
                                           unsigned cb, const char* Vb, T* Z, int64_t D, int zw) {
  T b[4][4];
#pragma unroll
  for (int q = 0; q < 4; q++) {
    // a core without allowed pairs has written no list this batch: no loads for it
    if (d[q] == 0) continue;  // uniform
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const unsigned o = Rv[q][4 * j + kq];
      b[q][j] = *reinterpret_cast<const T*>(Vb + ((o & ~1u) + cb));
    }
  }
#pragma unroll
  for (int q = 0; q < 4; q++) {
    if (d[q] == 0) continue;  // uniform
    const int KS = (d[q] + 3) >> 2;
    const int tb = (Pi[q][c] & 255) * HW;
    typename Mfma<T>::acc acc = {0, 0, 0, 0};
#pragma unroll
    for (int j = 0; j < 4; j++) {
      if (j < KS) {
        const int kk = 4 * j + kq;
        acc = Mfma<T>::run(Hs[tb + (Pi[q][kk] & 255)], flip_if(b[q][j], Rv[q][kk] & 1u), acc);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; v++) {
      const int i = Mfma<T>::row(kq, v);
      const unsigned t = Rt[q][i];
      const int p = Pi[q][i];
      if (i < d[q] && cok)
        __builtin_nontemporal_store(flip_if((T)acc[v], (unsigned)(p >> 8) & 1u), Z + ((int64_t)(p >> 9) * D + t) * zw + c);
    }
  }
}

// One work item: up to PN_TPB cores of one (2M, parity) group and one pair block (cores staged in
// LDS); each wavefront takes every fourth core, four at a time, with the rank-table lookups of its
// next four issued one batch ahead. Lists per core: V byte offset | source sign, target index,
// pair index | sign << 8 | slot << 9; padded to 64 entries with a valid row and the zero pair.
template <class T>
__global__ __launch_bounds__(256, 4) void fly_tile_kernel(FlyTileArgs<T> a) {
  extern __shared__ __align__(16) char hs_[];
  T* Hs = reinterpret_cast<T*>(hs_);
  __shared__ int Ps[PN_MAXPAIR];
  __shared__ uint64_t Lc[PN_TPB];
  __shared__ unsigned Rv[4][4][64];
  __shared__ unsigned Rt[4][4][64];
  __shared__ int Pi[4][4][64];
  const int item = pn_xcd_item(blockIdx.x, a.nitems);
  if (item >= a.nitems) return;
  const int4 it = a.items[item];
  const int k = a.rect[2 * it.x], sk = a.rect[2 * it.x + 1];
  const int q0 = a.pr_off[k], D2 = a.pr_off[k + 1] - q0, HW = D2 + 1;
  const T* hg = a.hb + a.hb_off[k];
  for (int i = threadIdx.x / 64; i < HW; i += 4)
    for (int j = threadIdx.x % 64; j < HW; j += 64) Hs[i * HW + j] = (i < D2 && j < D2) ? hg[i * D2 + j] : T(0);
  for (int e = threadIdx.x; e < D2; e += 256) Ps[e] = a.pr_ab[q0 + e];
  for (int e = threadIdx.x; e < it.z; e += 256) Lc[e] = a.cw[it.y + e];
  __syncthreads();
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int c = l & 15, kq = l >> 4;
  const bool cok = c < a.cval;
  const unsigned cb = (unsigned)(a.c0 + min(c, a.cval - 1)) * (unsigned)sizeof(T);
  const int lp = min(l, D2 - 1);
  const int ab = Ps[lp], sa = ab & 255, sb = ab >> 8;  // sa < sb
  const int st = a.sstart[sk];
  const int* bk = a.base + ((int64_t)sk << a.half);
  const uint64_t lmask = (1ull << a.half) - 1, pair = (1ull << sa) | (1ull << sb);
  const char* Vb = reinterpret_cast<const char*>(a.V);
  const int n = it.z;
  // target index of pair l on core j (0 when not allowed), its lookups issued now
  auto target = [&](int j) __attribute__((always_inline)) {
    if (j >= n) return 0;
    const uint64_t L = Lc[j];
    if (l >= D2 || (L & pair) != 0) return 0;
    const uint64_t x = L | pair;
    return st + bk[x & lmask] + a.rank[x >> a.half];
  };
  int tn[4];
#pragma unroll
  for (int q = 0; q < 4; q++) tn[q] = target(w + 4 * q);
  for (int j0 = w; j0 < n; j0 += 16) {
    int tc[4], d[4];
#pragma unroll
    for (int q = 0; q < 4; q++) tc[q] = tn[q];
#pragma unroll
    for (int q = 0; q < 4; q++) tn[q] = target(j0 + 16 + 4 * q);
    bool big = false;
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const int j = j0 + 4 * q;
      const uint64_t L = j < n ? Lc[j] : ~0ull;
      const bool ok = l < D2 && (L & pair) == 0;
      const uint64_t mask = __ballot(ok);
      d[q] = __popcll(mask);
      big = big || d[q] > 16;
      if (d[q] == 0) continue;  // uniform
      const int below = __popcll(mask & ((1ull << l) - 1));
      const int t = tc[q];
      const int lead = __builtin_amdgcn_readlane(t, __builtin_ctzll(mask));
      if (ok) {
        const int pa = __popcll(L & ((1ull << sa) - 1)), pb = __popcll(L & ((1ull << sb) - 1)) + 1;
        const unsigned sg = (unsigned)((pa + pb + 1) & 1);  // sigma(L, a) sigma(L, b)
        Rv[w][q][below] = (unsigned)t * (unsigned)a.vrow | sg;
        Rt[w][q][below] = (unsigned)t;
        Pi[w][q][below] = l | (int)(sg << 8) | ((pb * (pb - 1) / 2 + pa) << 9);
      } else {
        const int pad = d[q] + l - below;
        Rv[w][q][pad] = (unsigned)lead * (unsigned)a.vrow;
        Pi[w][q][pad] = D2;
      }
    }
    __builtin_amdgcn_wave_barrier();
    if (!big) {
      fly_batch4<T>(Hs, Rv[w], Rt[w], Pi[w], d, HW, c, kq, cok, cb, Vb, a.Z, a.D, a.zw);
    } else {
#pragma unroll
      for (int q = 0; q < 4; q++) {
        if (d[q] > 32) fly_product<T, 4>(Hs, Rv[w][q], Rt[w][q], Pi[w][q], d[q], HW, c, kq, cok, cb, Vb, a.Z, a.D, a.zw);
        else if (d[q] > 0)
          fly_product<T, 2>(Hs, Rv[w][q], Rt[w][q], Pi[w][q], d[q], HW, c, kq, cok, cb, Vb, a.Z, a.D, a.zw);
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// W[t][c0 + c] = (single-particle energies of t) V[t][c0 + c] + the slots of t in slot order
// (internal order, packed nb); targets outside a truncated space (mask 0) get 0
template <class T>
__global__ void fly_finalize_kernel(const T* __restrict__ V, T* __restrict__ W, int nb, const T* __restrict__ Z, int S,
                                    int64_t D, int zw, int c0, int cval, const uint64_t* words, const T* e,
                                    const double* mask, const int* perm, const int64_t* soff, const int* sstart,
                                    int nsec) {
  const int64_t n = D * zw;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(q % zw);
    if (c >= cval) continue;
    const int64_t t = q / zw;
    T* wt = W + t * nb + c0 + c;
    if (mask) {
      int k = 0;
      while (k + 1 < nsec && t >= sstart[k + 1]) k++;
      if (mask[soff[k] + perm[t]] == 0.0) {
        *wt = T(0);
        continue;
      }
    }
    T s = T(0);
    for (uint64_t x = words[t]; x; x &= x - 1) s += e[__builtin_ctzll(x)];
    s *= V[t * nb + c0 + c];
    const T* z = Z + t * zw + c;
    int k = 0;
    for (; k + 8 <= S; k += 8) {
      T zq[8];
#pragma unroll
      for (int j = 0; j < 8; j++) zq[j] = __builtin_nontemporal_load(z + (int64_t)(k + j) * D * zw);
#pragma unroll
      for (int j = 0; j < 8; j++) s += zq[j];
    }
    for (; k < S; k++) s += __builtin_nontemporal_load(z + (int64_t)k * D * zw);
    *wt = s;
  }
}

}  // namespace

// ------------------------------------------------------------------ one species: host tables and launch
void build_fly_tiles(Model& m) {
  FlyTiles& F = m.flyt;
  F.on = false;
  F.z.release();
  const char* env = std::getenv("TRBL_PN_TILES");
  if (env && env[0] == '0') return;
  const Species& SP = m.sp[m.fly_s];
  const int ns = m.ns, npart = SP.npart, tj = m.cl.tjmax;
  if (npart < 2) return;
  const std::vector<MTerm>& terms = m.fly_s == 1 ? m.terms_nn : m.terms_pp;
  auto stpar = [&](int st) { return (m.orbits[m.st_orb[st]].l & 1) ? 1 : 0; };  // 1: odd
  // pair blocks by (2M, parity) of the pair, pairs a < b
  std::map<std::pair<int, int>, int> kid;
  std::vector<std::vector<int>> pairs;
  std::vector<int> pid(ns * ns, -1), pk(ns * ns, -1);
  for (int a0 = 0; a0 < ns; a0++)
    for (int b0 = a0 + 1; b0 < ns; b0++) {
      const std::pair<int, int> key{m.st_tm[a0] + m.st_tm[b0], stpar(a0) ^ stpar(b0)};
      auto itk = kid.find(key);
      if (itk == kid.end()) {
        itk = kid.emplace(key, (int)pairs.size()).first;
        pairs.emplace_back();
      }
      pk[a0 * ns + b0] = itk->second;
      pid[a0 * ns + b0] = (int)pairs[itk->second].size();
      pairs[itk->second].push_back(a0 | (b0 << 8));
    }
  const int nk = (int)pairs.size();
  int maxp = 0;
  for (auto& v : pairs) maxp = std::max(maxp, (int)v.size());
  if (maxp > PN_MAXPAIR) return;
  std::vector<int> pr_off(nk + 1, 0), pr_ab, hb_off(nk + 1, 0);
  for (int k = 0; k < nk; k++) {
    pr_off[k + 1] = pr_off[k] + (int)pairs[k].size();
    hb_off[k + 1] = hb_off[k] + (int)(pairs[k].size() * pairs[k].size());
    pr_ab.insert(pr_ab.end(), pairs[k].begin(), pairs[k].end());
  }
  std::vector<double> hb(hb_off[nk], 0.0);
  for (const MTerm& t : terms) {  // c+_a c+_b c_d c_c, a < b, c < d
    TRBL_REQUIRE(t.a < t.b && t.c < t.d, TRBL_E_INVALID, "identical-particle term not in canonical order");
    const int k = pk[t.a * ns + t.b];
    TRBL_REQUIRE(k == pk[t.c * ns + t.d], TRBL_E_INVALID, "two-body term breaks M or parity conservation");
    const int D2 = (int)pairs[k].size();
    hb[hb_off[k] + pid[t.a * ns + t.b] * D2 + pid[t.c * ns + t.d]] += t.h;
  }
  // cores: (n - 2)-subsets grouped by (2M, parity); only groups whose pairs reach a stored sector
  const int nc = npart - 2;
  if (binom(ns, nc) > (int64_t)1 << 27) return;
  std::map<std::pair<int, int>, int> secid;
  for (int q = 0; q < (int)SP.sectors.size(); q++) secid[{SP.sectors[q].twoM, SP.sectors[q].par < 0 ? 1 : 0}] = q;
  std::map<std::pair<int, int>, std::vector<uint64_t>> by;
  auto visit = [&](uint64_t w) {
    int tm = 0, par = 0;
    for (uint64_t x = w; x; x &= x - 1) {
      const int st = __builtin_ctzll(x);
      tm += m.st_tm[st];
      par ^= stpar(st);
    }
    by[{tm, par}].push_back(w);
  };
  if (nc == 0) {
    visit(0);
  } else {
    uint64_t w = (1ull << nc) - 1;
    const uint64_t limit = ns == 64 ? 0ull : (1ull << ns);
    while (true) {
      visit(w);
      const uint64_t lo = w & (~w + 1), hi = w + lo;
      if (hi == 0) break;
      const uint64_t nw = (((hi ^ w) >> 2) / lo) | hi;
      if ((ns < 64 && nw >= limit) || nw <= w) break;
      w = nw;
    }
  }
  std::vector<uint64_t> cw;
  std::vector<int> rect, items;
  for (auto& kv : by) {
    std::vector<std::pair<int, int>> rs;  // (pair block, sector)
    for (const auto& sv : secid) {
      const int tmp = sv.first.first - kv.first.first, parp = sv.first.second ^ kv.first.second;
      auto itk = kid.find({tmp, parp});
      if (itk != kid.end()) rs.push_back({itk->second, sv.second});
    }
    if (rs.empty()) continue;
    // cores in the order of the internal numbering (low part of the m-states first): consecutive
    // cores then reach targets and sources in nearby ranges of V and of the slots
    const uint64_t lm = (1ull << m.fly_half) - 1;
    std::sort(kv.second.begin(), kv.second.end(), [&](uint64_t x, uint64_t y) {
      return (x & lm) != (y & lm) ? (x & lm) < (y & lm) : (x >> m.fly_half) < (y >> m.fly_half);
    });
    const int c0 = (int)cw.size();
    cw.insert(cw.end(), kv.second.begin(), kv.second.end());
    const int n = (int)kv.second.size();
    for (const auto& r : rs) {
      const int ri = (int)(rect.size() / 2);
      rect.insert(rect.end(), {r.first, r.second});
      for (int q = 0; q < n; q += PN_TPB) items.insert(items.end(), {ri, c0 + q, std::min(PN_TPB, n - q), 0});
    }
  }
  if (items.empty()) return;
  TRBL_REQUIRE(items.size() / 4 < ((size_t)1 << 31) / 256, TRBL_E_INVALID, "too many cores for one launch");
  const int S = npart * (npart - 1) / 2;
  const int zw = 8;  // slot rows of 8 columns; wider products run in tiles of 8
  const size_t zbytes = (size_t)S * (size_t)m.dim * zw * sizeof(double);
  size_t fr = 0, tot = 0;
  TRBL_HIP(hipMemGetInfo(&fr, &tot));
  if (zbytes > fr / 4 || (double)m.dim * 64 * 8 >= 4294967296.0 || (double)S * m.dim >= 4294967296.0) return;
  F.S = S;
  F.zw = zw;
  F.max_pairs = maxp;
  F.items = (int64_t)(items.size() / 4);
  F.cw.upload(cw);
  F.pr_off.upload(pr_off);
  F.pr_ab.upload(pr_ab);
  F.hb_off.upload(hb_off);
  F.hb.upload(hb);
  F.hb32.upload(std::vector<float>(hb.begin(), hb.end()));
  F.rect.upload(rect);
  F.items_buf.upload(items);
  F.z.alloc(zbytes);
  F.on = true;
}

template <class T>
void launch_fly_tiles(const Model& m, int nb, const T* Vint, T* Wint, const double* mask, hipStream_t s) {
  const FlyTiles& F = m.flyt;
  const DeviceTables& d = m.dt;
  FlyTileArgs<T> a{};
  a.V = Vint;
  a.Z = F.z.as<T>();
  a.zw = F.zw;
  a.ns = m.ns;
  a.half = m.fly_half;
  a.D = (int)m.dim;
  a.vrow = (int)(nb * sizeof(T));
  a.cw = F.cw.as<uint64_t>();
  a.base = d.fly_base.as<int>();
  a.rank = d.fly_rank.as<int>();
  a.sstart = d.fly_sstart.as<int>();
  a.pr_off = F.pr_off.as<int>();
  a.pr_ab = F.pr_ab.as<int>();
  a.hb_off = F.hb_off.as<int>();
  a.hb = (sizeof(T) == 8 ? F.hb : F.hb32).as<T>();
  a.rect = F.rect.as<int>();
  a.items = F.items_buf.as<int4>();
  a.nitems = (int)F.items;
  const unsigned grid = (unsigned)((F.items + 7) / 8 * 8);
  const size_t shm = (size_t)(F.max_pairs + 1) * (F.max_pairs + 1) * sizeof(T);
  const int nsec = (int)m.sp[m.fly_s].sectors.size();
  for (int c0 = 0; c0 < nb; c0 += F.zw) {
    a.c0 = c0;
    a.cval = std::min(F.zw, nb - c0);
    hipLaunchKernelGGL(fly_tile_kernel<T>, dim3(grid), dim3(256), shm, s, a);
    hipLaunchKernelGGL(fly_finalize_kernel<T>, dim3(elementwise_grid(m.dim * F.zw)), dim3(256), 0, s, Vint, Wint, nb,
                       (const T*)a.Z, F.S, m.dim, F.zw, c0, a.cval, d.fly_wint.as<uint64_t>(),
                       (sizeof(T) == 8 ? d.fly_e64 : d.fly_e32).as<T>(), mask, d.fly_perm.as<int>(),
                       d.fly_soff.as<int64_t>(), d.fly_sstart.as<int>(), nsec);
  }
  TRBL_HIP(hipGetLastError());
}
template void launch_fly_tiles<double>(const Model&, int, const double*, double*, const double*, hipStream_t);
template void launch_fly_tiles<float>(const Model&, int, const float*, float*, const double*, hipStream_t);

}  // namespace trbl
