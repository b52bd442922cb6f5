// Proton-neutron part of the block H.V (App. B) as dense pair blocks on the matrix cores.
//
// Every pn term c+_a(p) c+_b(n) c_d(n) c_c(p) moves one proton (c -> a) and one neutron (d -> b).
// Acting on a basis state it keeps the other protons, a core K_p of n_prot - 1 particles, and the
// other neutrons, a core K_n. Take the pair states (x, u), x a proton m-state and u a neutron
// m-state, grouped by their total 2m. For a fixed core pair (K_p, K_n) the states K_p+x, K_n+u
// with x outside K_p and u outside K_n, and 2m(x) + 2m(u) = 2M - 2M(K_p) - 2M(K_n), are linked
// by the pn terms as a dense symmetric block: the m-scheme pn matrix H_M[(x,u)][(y,v)] of that
// pair 2m, restricted to the allowed pairs. The Jordan-Wigner sign of c+_x c_y on K_p+y is
// sigma(K_p, x) sigma(K_p, y), sigma(K, s) = (-1)^(occupied states of K below s), and the same on
// the neutron side, so the sign of an element factorises into a target and a source sign.
//
// Each term is counted in exactly one core pair (the core is the set of spectator nucleons;
// a = c is a proton number operator, and its core is the target minus a), so the pn part of W is
//   W[t] += sum over the n_prot * n_neut core pairs of t of  s_t (H_M (s V))[t].
// A wavefront takes one core pair: it lists the allowed pairs with a ballot, gathers the source
// rows (16 columns, one 128-byte line each) with their signs, multiplies by the block of H_M on
// the matrix cores (v_mfma_f64_16x16x4f64), and writes each target row into the slot named by
// the positions of x in the target's proton word and of u in its neutron word. Every slot of
// every basis state is written exactly once per product, so the second kernel sums the slots
// into W in a fixed order: no atomics, and the result does not depend on scheduling.
#include <algorithm>
#include <cstdlib>
#include <map>

#include "tilecore.h"

namespace trbl {

using namespace tiles;

namespace {

template <class T>
struct PNTileArgs {
  const T* V;
  T* Z;
  int c0, cval;  // column tile: first column, valid columns (<= 16)
  int ns, nneut, D, vrow;  // vrow: bytes per row of V
  const int* rkp;  // [core * ns + state]: position << 24 | local index of core + state, -1 inside
  const int* rkn;
  const int* blk_off;  // block offsets (the tables are used only while D < 2^31)
  const int* blk_dn;
  const int* pr_off;
  const int* pr_xu;
  const int* hb_off;
  const T* hb;
  const int* rect;    // per rectangle: pair block, first entry of its list in rblk
  const int* rblk;    // per rectangle and pair: block of the target's sectors, -1 if none
  const int4* items;  // per work item: rectangle, proton core, first neutron core, count
  int nitems;
};

// The product of one core pair: Z rows of its d allowed targets = (staged block) x (signed source
// rows), DTM row tiles of 16 targets at most (d <= 16 DTM); sources k = 4 ks + l / 16 in groups
// of 8 steps whose loads are issued together.
template <class T, int DTM>
__device__ __forceinline__ void tile_mfma(const T* Hs, const unsigned* Rv, const int* Pi, int h, int KS, int DT,
                                          const int (&tb)[DTM], int kq, const T (&bop)[8],
                                          typename Mfma<T>::acc (&acc)[DTM]) {
#pragma unroll
  for (int j = 0; j < 8; j++) {
    if (8 * h + j < KS) {
      const int kk = 4 * (8 * h + j) + kq;
      const T b = flip_if(bop[j], Rv[kk] & 1u);
      const int pk = Pi[kk];
      T av[DTM];
#pragma unroll
      for (int mt = 0; mt < DTM; mt++) av[mt] = Hs[tb[mt] + pk];
#pragma unroll
      for (int mt = 0; mt < DTM; mt++)
        if (mt < DT) acc[mt] = Mfma<T>::run(av[mt], b, acc[mt]);
    }
  }
}

template <class T, int DTM>
__device__ __forceinline__ void tile_init(const int* Pi, int HW, int c, int (&tb)[DTM],
                                          typename Mfma<T>::acc (&acc)[DTM]) {
#pragma unroll
  for (int mt = 0; mt < DTM; mt++) {
    tb[mt] = Pi[16 * mt + c] * HW;
    acc[mt] = typename Mfma<T>::acc{0, 0, 0, 0};
  }
}

template <class T, int DTM>
__device__ __forceinline__ void tile_store(const unsigned* Rz, int d, int DT, int c, int kq, bool cok, char* Zb,
                                           const typename Mfma<T>::acc (&acc)[DTM]) {
#pragma unroll
  for (int mt = 0; mt < DTM; mt++) {
    if (mt < DT) {
#pragma unroll
      for (int v = 0; v < 4; v++) {
        const int i = 16 * mt + Mfma<T>::row(kq, v);
        const unsigned z = Rz[i];
        if (i < d && cok)
          __builtin_nontemporal_store(flip_if((T)acc[mt][v], z & 1u),
                                      reinterpret_cast<T*>(Zb + ((z & ~63u) + (unsigned)c * (unsigned)sizeof(T))));
      }
    }
  }
}

template <class T, int DTM>
__device__ __forceinline__ void tile_product(const T* Hs, const unsigned* Rv, const unsigned* Rz, const int* Pi, int d,
                                             int HW, int c, int kq, bool cok, unsigned cb, const char* Vb, char* Zb) {
  const int KS = (d + 3) >> 2, DT = (d + 15) >> 4;
  int tb[DTM];
  typename Mfma<T>::acc acc[DTM];
  tile_init<T, DTM>(Pi, HW, c, tb, acc);
#pragma unroll
  for (int h = 0; h < DTM / 2; h++) {
    T bop[8];
    tile_loads<T>(Rv, h, kq, cb, Vb, bop);
    tile_mfma<T, DTM>(Hs, Rv, Pi, h, KS, DT, tb, kq, bop, acc);
    __builtin_amdgcn_sched_barrier(0);
  }
  tile_store<T, DTM>(Rz, d, DT, c, kq, cok, Zb, acc);
}

// Two core pairs of at most 32 allowed pairs each: the loads of both are issued before the
// products, so a wavefront keeps twice the rows in flight.
template <class T>
__device__ __forceinline__ void tile_product2(const T* Hs, const unsigned* RvA, const unsigned* RzA, const int* PiA,
                                              int dA, const unsigned* RvB, const unsigned* RzB, const int* PiB, int dB,
                                              int HW, int c, int kq, bool cok, unsigned cb, const char* Vb, char* Zb) {
  const int KSA = (dA + 3) >> 2, DTA = (dA + 15) >> 4, KSB = (dB + 3) >> 2, DTB = (dB + 15) >> 4;
  T bA[8], bB[8];
  tile_loads<T>(RvA, 0, kq, cb, Vb, bA);
  tile_loads<T>(RvB, 0, kq, cb, Vb, bB);
  int tbA[2], tbB[2];
  typename Mfma<T>::acc aA[2], aB[2];
  tile_init<T, 2>(PiA, HW, c, tbA, aA);
  tile_init<T, 2>(PiB, HW, c, tbB, aB);
  tile_mfma<T, 2>(Hs, RvA, PiA, 0, KSA, DTA, tbA, kq, bA, aA);
  tile_store<T, 2>(RzA, dA, DTA, c, kq, cok, Zb, aA);
  tile_mfma<T, 2>(Hs, RvB, PiB, 0, KSB, DTB, tbB, kq, bB, aB);
  tile_store<T, 2>(RzB, dB, DTB, c, kq, cok, Zb, aB);
}

// One work item: a proton core K_p and up to PN_TPB neutron cores of one (2M, parity) group; the
// four wavefronts take every fourth core pair. Per core pair the allowed pairs are listed in LDS
// (V byte offset | source sign, slot byte offset | target sign, pair index); the list is padded
// to 64 entries with a valid row and the pair index D2, whose row and column of the staged block
// are zero, so the products need no masks.
template <class T>
__global__ __launch_bounds__(256, 4) void pn_tile_kernel(PNTileArgs<T> a) {
  extern __shared__ __align__(16) char hs_[];  // (widest block + 1)^2 values
  T* Hs = reinterpret_cast<T*>(hs_);
  __shared__ int Po[PN_MAXPAIR];  // per pair: offset of its block (-1: no block)
  __shared__ int Pd[PN_MAXPAIR];  // per pair: neutron sector size of its block
  __shared__ int Ps[PN_MAXPAIR];  // per pair: x | u << 8
  __shared__ unsigned Rv[4][2][64];
  __shared__ unsigned Rz[4][2][64];
  __shared__ int Pi[4][2][64];
  const int item = pn_xcd_item(blockIdx.x, a.nitems);
  if (item >= a.nitems) return;
  const int4 it = a.items[item];
  const int k = a.rect[2 * it.x], rb0 = a.rect[2 * it.x + 1];
  const int q0 = a.pr_off[k], D2 = a.pr_off[k + 1] - q0, HW = D2 + 1;
  const T* hg = a.hb + a.hb_off[k];
  for (int i = threadIdx.x / 64; i < HW; i += 4)
    for (int j = threadIdx.x % 64; j < HW; j += 64) Hs[i * HW + j] = (i < D2 && j < D2) ? hg[i * D2 + j] : T(0);
  for (int e = threadIdx.x; e < D2; e += 256) {
    Ps[e] = a.pr_xu[q0 + e];
    const int b = a.rblk[rb0 + e];
    Po[e] = b >= 0 ? a.blk_off[b] : -1;
    Pd[e] = b >= 0 ? a.blk_dn[b] : 0;
  }
  __syncthreads();
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int c = l & 15, kq = l >> 4;
  const bool cok = c < a.cval;
  // column byte; beyond the tile: a valid column
  const unsigned cb = (unsigned)(a.c0 + min(c, a.cval - 1)) * (unsigned)sizeof(T);
  const int lp = min(l, D2 - 1);
  const int xu = Ps[lp], us = xu >> 8;
  const int poff = Po[lp], pdn = Pd[lp];
  const int rp = a.rkp[it.y * a.ns + (xu & 255)];  // the proton core is fixed for the item
  const bool lok = l < D2 && poff >= 0 && rp >= 0;
  const int bp = rp >> 24;
  const int rowp = poff + (rp & 0xFFFFFF) * pdn;
  const char* Vb = reinterpret_cast<const char*>(a.V);
  char* Zb = reinterpret_cast<char*>(a.Z);
  // the list of one core pair (neutron core entry rn) into buffer q; returns its allowed pairs
  auto list = [&](int rn, int q) __attribute__((always_inline)) {
    const bool ok = lok && rn >= 0;
    const uint64_t mask = __ballot(ok);
    const int d = __popcll(mask);
    if (d == 0) return 0;  // uniform
    const int below = __popcll(mask & ((1ull << l) - 1));
    const int bn = rn >> 24;
    const int row = rowp + (rn & 0xFFFFFF);
    const unsigned sg = (unsigned)((bp + bn) & 1);
    const int lead = __builtin_amdgcn_readlane(row, __builtin_ctzll(mask));
    if (ok) {
      Rv[w][q][below] = (unsigned)row * (unsigned)a.vrow | sg;
      Rz[w][q][below] = ((unsigned)((bp * a.nneut + bn) * a.D + row) << Mfma<T>::ZSHIFT) | sg;
      Pi[w][q][below] = l;
    } else {  // padding: a valid row, the zero pair
      const int pad = d + l - below;
      Rv[w][q][pad] = (unsigned)lead * (unsigned)a.vrow;
      Pi[w][q][pad] = D2;
    }
    return d;
  };
  int cn = it.z + w;
  const int cend = it.z + it.w;
  // neutron-core entries of the next two core pairs of this wavefront, loaded one step ahead
  int rnA = cn < cend ? a.rkn[cn * a.ns + us] : -1;
  int rnB = cn + 4 < cend ? a.rkn[(cn + 4) * a.ns + us] : -1;
  for (; cn < cend; cn += 8) {
    const int rA = rnA, rB = rnB;
    const bool hasB = cn + 4 < cend;
    if (cn + 8 < cend) rnA = a.rkn[(cn + 8) * a.ns + us];
    if (cn + 12 < cend) rnB = a.rkn[(cn + 12) * a.ns + us];
    const int dA = list(rA, 0);
    const int dB = hasB ? list(rB, 1) : 0;
    // the lists are written and read by this wavefront only: LDS operations of one wavefront
    // complete in order, so only the compiler must keep them in place
    __builtin_amdgcn_wave_barrier();
    if (dA > 0 && dA <= 32 && dB > 0 && dB <= 32) {
      tile_product2<T>(Hs, Rv[w][0], Rz[w][0], Pi[w][0], dA, Rv[w][1], Rz[w][1], Pi[w][1], dB, HW, c, kq, cok, cb, Vb,
                       Zb);
    } else {
      if (dA > 32) tile_product<T, 4>(Hs, Rv[w][0], Rz[w][0], Pi[w][0], dA, HW, c, kq, cok, cb, Vb, Zb);
      else if (dA > 0) tile_product<T, 2>(Hs, Rv[w][0], Rz[w][0], Pi[w][0], dA, HW, c, kq, cok, cb, Vb, Zb);
      if (dB > 32) tile_product<T, 4>(Hs, Rv[w][1], Rz[w][1], Pi[w][1], dB, HW, c, kq, cok, cb, Vb, Zb);
      else if (dB > 0) tile_product<T, 2>(Hs, Rv[w][1], Rz[w][1], Pi[w][1], dB, HW, c, kq, cok, cb, Vb, Zb);
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// W[t][c0 + c] += sum of the S slots of t, in slot order
template <class T>
__global__ void pn_reduce_kernel(const T* __restrict__ Z, int S, int64_t D, T* __restrict__ W, int64_t ldw, int c0,
                                 int cval) {
  const int64_t n = D * 16;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e & 15);
    if (c >= cval) continue;
    const int64_t t = e >> 4;
    T s = T(0);
    for (int k = 0; k < S; k++) s += __builtin_nontemporal_load(Z + ((int64_t)k * D + t) * 16 + c);
    W[t * ldw + c0 + c] += s;
  }
}

}  // namespace

void build_pn_tiles(Model& m) {
  PNTiles& T = m.pn;
  T.on = false;
  T.z.release();
  const char* env = std::getenv("TRBL_PN_TILES");
  if (env && env[0] == '0') return;
  T.force = env && env[0] == '2';
  if (m.fly || m.n_prot == 0 || m.n_neut == 0) return;
  const int ns = m.ns, tj = m.cl.tjmax;
  const int nk = 2 * tj + 1;
  // pair blocks by pair 2m: (x, u) with 2m(x) + 2m(u) = 2 (k - tj)
  std::vector<std::vector<int>> pairs(nk);
  std::vector<int> pid(ns * ns, -1);
  for (int x = 0; x < ns; x++)
    for (int u = 0; u < ns; u++) {
      const int k = (m.st_tm[x] + m.st_tm[u] + 2 * tj) / 2;
      pid[x * ns + u] = (int)pairs[k].size();
      pairs[k].push_back(x | (u << 8));
    }
  int maxp = 0;
  for (auto& v : pairs) maxp = std::max(maxp, (int)v.size());
  if (maxp > PN_MAXPAIR) return;
  // Every slot row (16 values written, then read back) carries the products of one core pair:
  // on average about L = (pair-weighted mean block size) x (share of the proton states outside a
  // proton core) x (the same for neutrons) source pairs. With few of them the slot traffic costs
  // more than the elements it carries: pf 3+3, 4+4 and 5+3 (L = 31 to 35) run 1.0 to 2.3 times
  // faster on the pair blocks (FP64 at 8 and 16 columns, FP32 at 16), sd 5+5 and 6+6 (L = 9.0
  // and 6.9) up to 2.9 times slower, sd 4+4 (L = 11.4) slower at 8 columns and faster at 16. The
  // pair blocks are taken from L = 16 on (TRBL_PN_TILES=2 takes them regardless).
  {
    double n1 = 0.0, n2 = 0.0;
    for (auto& v : pairs) {
      n1 += (double)v.size();
      n2 += (double)v.size() * (double)v.size();
    }
    const double L = n2 / n1 * (double)(ns - (m.n_prot - 1)) / ns * (double)(ns - (m.n_neut - 1)) / ns;
    if (L < 16.0 && !T.force) return;
  }
  std::vector<int> pr_off(nk + 1, 0), pr_xu, hb_off(nk + 1, 0);
  for (int k = 0; k < nk; k++) {
    pr_off[k + 1] = pr_off[k] + (int)pairs[k].size();
    hb_off[k + 1] = hb_off[k] + (int)(pairs[k].size() * pairs[k].size());
    pr_xu.insert(pr_xu.end(), pairs[k].begin(), pairs[k].end());
  }
  std::vector<double> hb(hb_off[nk], 0.0);
  for (const MTerm& t : m.terms_pn) {  // c+_a(p) c+_b(n) c_d(n) c_c(p): target pair (a, b), source pair (c, d)
    const int k = (m.st_tm[t.a] + m.st_tm[t.b] + 2 * tj) / 2;
    const int kc = (m.st_tm[t.c] + m.st_tm[t.d] + 2 * tj) / 2;
    TRBL_REQUIRE(k == kc, TRBL_E_INVALID, "pn term breaks M conservation");
    const int D2 = (int)pairs[k].size();
    hb[hb_off[k] + pid[t.a * ns + t.b] * D2 + pid[t.c * ns + t.d]] += t.h;
  }
  // cores of each species: all (N - 1)-subsets, grouped by (2M, parity)
  struct Group {
    int tm, par, start, count;
  };
  std::vector<Group> groups[2];
  std::vector<uint64_t> cw[2];
  std::vector<int> rk[2];
  std::map<std::pair<int, int>, int> secid[2];
  for (int s = 0; s < 2; s++) {
    const Species& S = m.sp[s];
    for (int q = 0; q < (int)S.sectors.size(); q++) secid[s][{S.sectors[q].twoM, S.sectors[q].par}] = q;
    const int nc = S.npart - 1;
    if (binom(ns, nc) > (1 << 21)) return;
    std::map<std::pair<int, int>, std::vector<uint64_t>> by;
    auto visit = [&](uint64_t w) {
      int tm = 0, ls = 0;
      for (uint64_t x = w; x; x &= x - 1) {
        const int st = __builtin_ctzll(x);
        tm += m.st_tm[st];
        ls += m.orbits[m.st_orb[st]].l;
      }
      by[{tm, (ls & 1) ? -1 : 1}].push_back(w);
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
    for (auto& kv : by) {
      groups[s].push_back({kv.first.first, kv.first.second, (int)cw[s].size(), (int)kv.second.size()});
      for (uint64_t w : kv.second) {
        cw[s].push_back(w);
        for (int st = 0; st < ns; st++) {
          if ((w >> st) & 1) {
            rk[s].push_back(-1);
            continue;
          }
          const auto it = S.index.find(w | (1ull << st));
          if (it == S.index.end()) {  // sector not stored: no block of the space holds it
            rk[s].push_back(-1);
            continue;
          }
          const int q = S.sector_of[it->second];
          const int loc = it->second - S.sectors[q].start;
          TRBL_REQUIRE(loc < (1 << 24), TRBL_E_INVALID, "sector too large for the pair-block tables");
          rk[s].push_back((__builtin_popcountll(w & ((1ull << st) - 1)) << 24) | loc);
        }
      }
    }
  }
  // block of (proton sector, neutron sector)
  const int nnsec = (int)m.sp[1].sectors.size();
  std::vector<int> bos(m.sp[0].sectors.size() * nnsec, -1);
  for (size_t b = 0; b < m.blocks.size(); b++) bos[m.blocks[b].psec * nnsec + m.blocks[b].nsec] = (int)b;
  auto stpar = [&](int st) { return (m.orbits[m.st_orb[st]].l & 1) ? -1 : 1; };
  // rectangles of core groups whose pair block reaches some block of the space
  std::vector<int> rect, rblk;
  std::vector<int> rect_of;  // per (proton group, neutron group): rectangle or -1
  for (const Group& gp : groups[0])
    for (const Group& gn : groups[1]) {
      rect_of.push_back(-1);
      const int tmp = m.twoM - gp.tm - gn.tm;
      if (tmp < -2 * tj || tmp > 2 * tj) continue;
      const int k = (tmp + 2 * tj) / 2;
      bool any = false;
      std::vector<int> pb;
      for (int xu : pairs[k]) {
        const int x = xu & 255, u = xu >> 8;
        auto ip = secid[0].find({gp.tm + m.st_tm[x], gp.par * stpar(x)});
        auto in = secid[1].find({gn.tm + m.st_tm[u], gn.par * stpar(u)});
        const int b = (ip != secid[0].end() && in != secid[1].end()) ? bos[ip->second * nnsec + in->second] : -1;
        pb.push_back(b);
        any = any || b >= 0;
      }
      if (!any) continue;
      rect_of.back() = (int)(rect.size() / 2);
      rect.insert(rect.end(), {k, (int)rblk.size()});
      rblk.insert(rblk.end(), pb.begin(), pb.end());
    }
  if (rect.empty()) return;
  // work items: per proton core, per neutron group with a rectangle, up to `chunk` neutron cores
  // (TRBL_PN_CHUNK: a tuning override). Items go to the XCDs in contiguous ranges, and the
  // cores of a group in runs of 16 consecutive (colex) cores: one neutron group after the other
  // for the 16 cores of a run, so that the items in flight on an XCD share more source rows
  // in its L2 (pf 4+4: FP64 H.V 3.39 against 3.46 ms with one core at a time; runs of 8, 12,
  // 20, 32, 64 and 128 gave 3.40 to 3.45 ms).
  int chunk = PN_TPB;
  if (const char* ev = std::getenv("TRBL_PN_CHUNK")) chunk = std::max(8, std::min(PN_TPB, std::atoi(ev)));
  constexpr int CORE_RUN = 16;
  std::vector<int> items;
  const int ngn = (int)groups[1].size();
  for (int ip = 0; ip < (int)groups[0].size(); ip++) {
    const int c_lo = groups[0][ip].start, c_hi = c_lo + groups[0][ip].count;
    for (int t0 = c_lo; t0 < c_hi; t0 += CORE_RUN)
      for (int in = 0; in < ngn; in++) {
        const int r = rect_of[ip * ngn + in];
        if (r < 0) continue;
        const Group& gn = groups[1][in];
        for (int cp = t0; cp < std::min(c_hi, t0 + CORE_RUN); cp++)
          for (int c0 = 0; c0 < gn.count; c0 += chunk)
            items.insert(items.end(), {r, cp, gn.start + c0, std::min(chunk, gn.count - c0)});
      }
  }
  TRBL_REQUIRE(items.size() / 4 < ((size_t)1 << 31) / 256, TRBL_E_INVALID, "too many core pairs for one launch");
  // the slot buffer: S slots of 16 FP64 columns per basis state, sized within a quarter of the
  // free device memory (larger spaces keep the jump-list kernel)
  const int S = m.n_prot * m.n_neut;
  const size_t zbytes = (size_t)S * (size_t)m.dim * 16 * sizeof(double);
  // 32-bit byte offsets in the kernel: the slot buffer and V (rows of at most 64 columns) must
  // stay below 4 GiB
  if ((double)zbytes >= 4294967296.0 || (double)m.dim * 64 * 8 >= 4294967296.0) return;
  size_t fr = 0, tot = 0;
  TRBL_HIP(hipMemGetInfo(&fr, &tot));
  if (zbytes > fr / 4) return;
  T.S = S;
  T.nk = nk;
  T.nrect = (int)(rect.size() / 2);
  T.ncore[0] = (int)cw[0].size();
  T.ncore[1] = (int)cw[1].size();
  T.max_pairs = maxp;
  T.tpb = PN_TPB;
  T.items = (int64_t)(items.size() / 4);
  T.cw[0].upload(cw[0]);
  T.cw[1].upload(cw[1]);
  T.rk[0].upload(rk[0]);
  T.rk[1].upload(rk[1]);
  T.pr_off.upload(pr_off);
  T.pr_xu.upload(pr_xu);
  T.hb_off.upload(hb_off);
  T.hb.upload(hb);
  std::vector<float> hb32(hb.begin(), hb.end());
  T.hb32.upload(hb32);
  T.rect.upload(rect);
  T.rblk.upload(rblk);
  T.item0.upload(items);
  std::vector<int> boff32(m.blocks.size());
  for (size_t b = 0; b < m.blocks.size(); b++) boff32[b] = (int)m.blocks[b].off;
  T.boff.upload(boff32);
  T.z.alloc(zbytes);
  if (!T.side) TRBL_HIP(hipStreamCreateWithFlags(&T.side, hipStreamNonBlocking));
  for (auto& e : T.ev)
    if (!e) TRBL_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  T.on = true;
}

template <class T>
void launch_pn_tiles(const Model& m, int nb, const T* V, int64_t ldv, T* W, int64_t ldw, hipStream_t s, bool reduce) {
  const PNTiles& P = m.pn;
  PNTileArgs<T> a{};
  a.V = V;
  a.Z = P.z.as<T>();
  a.ns = m.ns;
  a.nneut = m.n_neut;
  a.D = (int)m.dim;
  a.vrow = (int)(ldv * sizeof(T));
  a.rkp = P.rk[0].as<int>();
  a.rkn = P.rk[1].as<int>();
  a.blk_off = P.boff.as<int>();
  a.blk_dn = m.dt.blk_dn.as<int>();
  a.pr_off = P.pr_off.as<int>();
  a.pr_xu = P.pr_xu.as<int>();
  a.hb_off = P.hb_off.as<int>();
  a.hb = (sizeof(T) == 8 ? P.hb : P.hb32).as<T>();
  a.rect = P.rect.as<int>();
  a.rblk = P.rblk.as<int>();
  a.items = P.item0.as<int4>();
  a.nitems = (int)P.items;
  const unsigned grid = (unsigned)((P.items + 7) / 8 * 8);
  const size_t shm = (size_t)(P.max_pairs + 1) * (P.max_pairs + 1) * sizeof(T);
  // a wider product reuses the slot buffer per 16 columns, each tile summed into W in turn; with
  // reduce false (one tile) the own-row kernel sums it
  for (int c0 = 0; c0 < nb; c0 += 16) {
    a.c0 = c0;
    a.cval = std::min(16, nb - c0);
    hipLaunchKernelGGL(pn_tile_kernel<T>, dim3(grid), dim3(256), shm, s, a);
    if (reduce || c0 + 16 < nb)
      hipLaunchKernelGGL(pn_reduce_kernel<T>, dim3(elementwise_grid(m.dim * 16)), dim3(256), 0, s, (const T*)a.Z, P.S,
                         m.dim, W, ldw, c0, a.cval);
  }
  TRBL_HIP(hipGetLastError());
}
template void launch_pn_tiles<double>(const Model&, int, const double*, int64_t, double*, int64_t, hipStream_t, bool);
template void launch_pn_tiles<float>(const Model&, int, const float*, int64_t, float*, int64_t, hipStream_t, bool);

}  // namespace trbl
