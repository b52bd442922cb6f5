// Block H.V planning and launch (App. B), and device-side basis indexing (App. A).
// The H.V kernels themselves are in hv_kern.h, instantiated per precision in
// hv_f64.hip and hv_f32.hip.
#include <cstdlib>
#include <map>

#include "hv_kern.h"
#include "rank.h"

namespace trbl {

extern template void dispatch_hv<double>(HVArgs<double>&, const HVPlan&, hipStream_t, int, unsigned);
extern template void dispatch_hv<float>(HVArgs<float>&, const HVPlan&, hipStream_t, int, unsigned);

static int pow2ceil(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

static int rs_of(int C, size_t elt) { return elt == 8 ? (C >= 2 ? C + 2 : 2) : (C >= 4 ? C + 4 : 4); }

// LDS bytes per row buffer of the rows kernel: 24 KB and 36 KB leave room for two workgroups per
// CU; 144 KB is one buffer (staged and waited for at each step) for the widest source rows, so
// that 3,952-wide sectors take a 4-column FP64 (8-column FP32) tile instead of half that
constexpr size_t ROW_SMALL = 24 * 1024, ROW_MID = 36 * 1024, ROW_LARGE = 72 * 1024, ROW_XL = 144 * 1024;

static HVPlan& plan_for(const Model& m, int nb, size_t elt) {
  const int key = nb * 16 + (int)elt;
  auto it = m.hv_plans.find(key);
  if (it != m.hv_plans.end()) return *it->second;
  auto owned = std::make_unique<HVPlan>();
  HVPlan* P = owned.get();
  // 1024-wide workgroups leave 128 VGPRs per lane: narrower tiles there
  const int cmin = (int)(16 / elt), cmax = (elt == 8 ? 16 : 32) / (m.max_dn > 768 ? 2 : 1);
  int C = std::max(cmin, std::min(cmax, pow2ceil(nb)));
  if (const char* env = std::getenv("TRBL_HV_TILE")) {  // tuning override: a narrower power-of-two tile
    C = std::max(cmin, std::min(C, std::atoi(env)));
    while (C & (C - 1)) C &= C - 1;
  }
  // TRBL_HV_XL=0: tiles sized for the 72 KB double buffer only, for comparison
  static const size_t row_cap =
      std::getenv("TRBL_HV_XL") && std::atoi(std::getenv("TRBL_HV_XL")) == 0 ? ROW_LARGE : ROW_XL;
  // a row buffer holds the widest source row plus the zero rows of the rows kernel (one per
  // part of a 256-byte bank window)
  auto zrows = [&](int c) { return (size_t)std::max<size_t>(1, 256 / (c * elt)); };
  while (C > cmin && (m.max_dn + zrows(C)) * C * elt > row_cap) C >>= 1;
  TRBL_REQUIRE((m.max_dn + zrows(C)) * C * elt <= row_cap, TRBL_E_INVALID, "neutron sector too large for the LDS row tile");
  // the columns kernel stages whole proton columns: its own, possibly narrower, tile
  int Cc = C;
  while (Cc > cmin && (size_t)m.max_dp * rs_of(Cc, elt) * elt > 144 * 1024) Cc >>= 1;
  TRBL_REQUIRE((size_t)m.max_dp * rs_of(Cc, elt) * elt <= 144 * 1024 && Cc * 4 >= C, TRBL_E_INVALID,
               "proton sector too large for the LDS column tile");
  // one row of the pn coefficient table must fit the rows kernel's 8 KB coefficient area, and the
  // double-buffered rows kernel holds every neutron jump of a class in registers
  TRBL_REQUIRE(m.max_nj_class <= 32, TRBL_E_INVALID, "more than 32 neutron jumps of one class from one SD");
  TRBL_REQUIRE((size_t)m.max_hncol * elt <= 8192, TRBL_E_INVALID, "pn operator class too large for the LDS table");
  P->C = C;
  P->ntile = (nb + C - 1) / C;
  P->Cc = Cc;
  P->ntile_c = (nb + Cc - 1) / Cc;
  // rows kernel: one launch per (launch bound, row buffer) class of blocks. The row buffer
  // must hold the widest source row a block's proton jumps can reach.
  const int ncl = m.cl.nclass;
  std::map<std::pair<int, int>, std::vector<int>> members;
  for (size_t b = 0; b < m.blocks.size(); b++) {
    const int dn = m.blocks[b].dn;
    if (dn == 0 || m.blocks[b].dp == 0) continue;
    int widest = dn;
    for (int c = 0; c < ncl; c++) {
      const int sb = m.src_blk_host[b * ncl + c];
      if (sb >= 0) widest = std::max(widest, m.blocks[sb].dn);
    }
    const int nthr = std::min(1024, (dn + 63) / 64 * 64);
    const int ntb = nthr <= 256 ? 256 : nthr <= 768 ? 768 : 1024;
    const size_t need = (widest + zrows(C)) * C * elt;
    const int rb = need <= ROW_SMALL ? 24 : need <= ROW_MID ? 36 : need <= ROW_LARGE ? 72 : 144;
    members[{ntb, rb}].push_back((int)b);
  }
  for (auto& kv : members) {
    P->bins.push_back(std::make_unique<HVBin>());
    HVBin& B = *P->bins.back();
    int maxdn = 0;
    for (int b : kv.second) maxdn = std::max(maxdn, m.blocks[b].dn);
    B.ntb = kv.first.first;
    B.rb_kb = kv.first.second;
    B.nthr = std::min(1024, (maxdn + 63) / 64 * 64);
    // sectors wider than 1024: 2 or 4 targets per lane, so a staged source row serves up to
    // 4096 targets (TRBL_HV_MP=1: one target per lane and 1024-wide chunks, for comparison)
    static const int mp_cap = [] {
      const char* env = std::getenv("TRBL_HV_MP");
      return env ? std::max(1, std::atoi(env)) : 4;
    }();
    if (B.ntb == 1024 && B.rb_kb >= 72 && maxdn > 1024 && mp_cap > 1) {
      const int want = (maxdn > 2048 && mp_cap >= 4) ? 4 : 2;
      if (rows_mp_fits((size_t)C * elt, want)) B.mp = want;
    }
    // register-held neutron jumps per class: every one of them with one target per lane
    B.nr = B.mp > 1 ? 8 : (m.max_nj_class > 16 ? 32 : 16);
    B.nchunk = (maxdn + B.nthr * B.mp - 1) / (B.nthr * B.mp);
    std::vector<int64_t> i0(1, 0);
    for (int b : kv.second) i0.push_back(i0.back() + (int64_t)m.blocks[b].dp * P->ntile * B.nchunk);
    B.nblk = (int)kv.second.size();
    B.maxdn = maxdn;
    B.items = i0.back();
    TRBL_REQUIRE(B.items < (int64_t)1 << 31 && (B.items + 7) * B.nthr < (int64_t)1 << 32, TRBL_E_INVALID,
                 "problem too large for one launch");
    B.blocks.upload(kv.second);
    B.item0.upload(i0);
  }
  // columns kernel
  P->nthr_c = std::min(1024, std::max(64, (m.max_dp + 63) / 64 * 64));
  P->maxp_c = 1;
  while (P->maxp_c < 4 && P->nthr_c * P->maxp_c < m.max_dp) P->maxp_c <<= 1;
  P->nchunk_c = (m.max_dp + P->nthr_c * P->maxp_c - 1) / (P->nthr_c * P->maxp_c);
  std::vector<int64_t> c0(m.blocks.size() + 1, 0);
  for (size_t b = 0; b < m.blocks.size(); b++)
    c0[b + 1] = c0[b] + (int64_t)m.blocks[b].dn * P->ntile_c * P->nchunk_c;
  P->cols_items = c0.back();
  TRBL_REQUIRE(P->cols_items < (int64_t)1 << 31 && (P->cols_items + 7) * P->nthr_c < (int64_t)1 << 32,
               TRBL_E_INVALID, "problem too large for one launch");
  P->citem0.upload(c0);
  P->shm_c = ((size_t)m.max_dp * rs_of(Cc, elt) * elt + 15) / 16 * 16;
  m.hv_plans[key] = std::move(owned);
  return *P;
}

template <class T>
static HVArgs<T> make_args(const Model& m, int nb, const void* V, int64_t ldv, void* W, int64_t ldw) {
  HVArgs<T> a{};
  a.V = static_cast<const T*>(V);
  a.W = static_cast<T*>(W);
  a.ldv = ldv;
  a.ldw = ldw;
  a.nb = nb;
  a.nblocks = (int)m.blocks.size();
  a.ncl = m.cl.nclass;
  a.tjmax = m.cl.tjmax;
  a.nnum = m.n_neut <= 8 ? m.n_neut : 0;  // number operators merged only while they are register-held
  a.nn_total = m.nn_total;
  // DMA staging needs 16-byte aligned chunks and full column tiles (set again once C is known)
  a.dma = ((uintptr_t)V % 16 == 0) && ((size_t)ldv * sizeof(T)) % 16 == 0;
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
  a.pg_start = d.pg_start.as<int>();
  a.pg_desc = d.pg_desc.as<int>();
  a.nj_start = d.nj_start.as<int>();
  a.nj32 = d.nj32.as<uint32_t>();
  a.pg_cend = d.pg_cend.as<int>();
  a.nlane = d.nlane.as<int>();
  a.h_off = d.h_off.as<int>();
  a.h_ncol = d.h_ncol.as<int>();
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
  } else {
    a.pe_val = d.pe_v32.as<T>();
    a.ne_val = d.ne_v32.as<T>();
    a.h = d.h32.as<T>();
  }
  return a;
}

template <class T>
static void run_hv(const Model& m, int nb, const void* V, int64_t ldv, void* W, int64_t ldw, hipStream_t s) {
  HVPlan& P = plan_for(m, nb, sizeof(T));
  HVArgs<T> a = make_args<T>(m, nb, V, ldv, W, ldw);
  a.C = P.C;
  a.ntile = P.ntile;
  a.dma = a.dma && nb % P.C == 0;
  a.citem0 = P.citem0.as<int64_t>();
  // with the pair-block tables the rows and columns kernels write the identical-particle parts and
  // the pair blocks add the pn part
  // The pair blocks work on 16-column tiles, so narrow products cost nearly as much as 16
  // columns; below the measured crossover (pf 4+4: FP64 from 5 columns, FP32 from 9, or from 5 at
  // widths that are not a power of two, where the jump-list kernel stages rows without the DMA)
  // the jump-list kernel runs instead. TRBL_PN_TILES=2 at set-up takes the pair blocks at every width.
  const bool pow2 = (nb & (nb - 1)) == 0;
  const bool wide = sizeof(T) == 8 ? nb >= 5 : (nb >= 9 || (nb >= 5 && !pow2));
  bool own = m.pn.on && (wide || m.pn.force) && (double)m.dim * (double)ldv * sizeof(T) < 4294967296.0;
  for (const auto& B : P.bins) own = own && B->mp == 1;
  a.own = own ? 1 : 0;
  if (!own) {
    dispatch_hv<T>(a, P, s, 3, ~0u);
    return;
  }
  // With the pair blocks: the columns kernel writes the pp part into W on the model's side stream
  // while the pair-block kernel writes the pn slots; the own-row kernel then adds the nn part and,
  // when one 16-column tile covers the product, the slots; a wider product adds its slots in a
  // pass of its own at the end.
  const PNTiles& pn = m.pn;
  TRBL_HIP(hipEventRecord(pn.ev[0], s));
  TRBL_HIP(hipStreamWaitEvent(pn.side, pn.ev[0], 0));
  a.ppset = 1;
  dispatch_hv<T>(a, P, pn.side, 2, ~0u);
  TRBL_HIP(hipEventRecord(pn.ev[1], pn.side));
  const bool fused = P.C == 16 && nb <= 16;
  if (fused) {
    launch_pn_tiles<T>(m, nb, static_cast<const T*>(V), ldv, static_cast<T*>(W), ldw, s, false);
    a.zs = pn.S;
    a.zstride = m.dim * 16;
    a.zbuf = pn.z.p;
  }
  // the own-row bins write disjoint rows: the largest runs here, the others on the side stream
  // (after the columns kernel there, and after the pair blocks)
  TRBL_REQUIRE(P.bins.size() <= 32, TRBL_E_INVALID, "more own-row bins than the stream split takes");
  size_t big = 0;
  for (size_t i = 1; i < P.bins.size(); i++)
    if (P.bins[i]->items * P.bins[i]->nthr > P.bins[big]->items * P.bins[big]->nthr) big = i;
  const unsigned bigmask = 1u << big;
  TRBL_HIP(hipEventRecord(pn.ev[2], s));
  TRBL_HIP(hipStreamWaitEvent(pn.side, pn.ev[2], 0));
  dispatch_hv<T>(a, P, pn.side, 1, ~bigmask);
  TRBL_HIP(hipEventRecord(pn.ev[3], pn.side));
  TRBL_HIP(hipStreamWaitEvent(s, pn.ev[1], 0));
  dispatch_hv<T>(a, P, s, 1, bigmask);
  TRBL_HIP(hipStreamWaitEvent(s, pn.ev[3], 0));
  if (!fused) launch_pn_tiles<T>(m, nb, static_cast<const T*>(V), ldv, static_cast<T*>(W), ldw, s, true);
}

void prepare_hv_plans(const Model& m, int precision, const int* widths, int n) {
  if (m.fly) return;
  for (int k = 0; k < n; k++) (void)plan_for(m, widths[k], precision == TRBL_FP64 ? sizeof(double) : sizeof(float));
}

bool has_hv_plan(const Model& m, int precision, int nb) {
  if (m.fly) return false;
  const int key = nb * 16 + (precision == TRBL_FP64 ? (int)sizeof(double) : (int)sizeof(float));
  return m.hv_plans.find(key) != m.hv_plans.end();
}

void launch_apply(const Model& m, int precision, int nb, const void* V, int64_t ldv, void* W, int64_t ldw,
                  hipStream_t s) {
  TRBL_REQUIRE(m.has_h, TRBL_E_STATE, "no Hamiltonian set");
  TRBL_REQUIRE(nb >= 1 && nb <= 64, TRBL_E_INVALID, "nb must be 1..64");
  TRBL_REQUIRE(ldv >= nb && ldw >= nb, TRBL_E_INVALID, "leading dimension smaller than nb");
  TRBL_REQUIRE(V && W && V != W, TRBL_E_INVALID, "V and W must be distinct device buffers");
  if (m.fly) {
    launch_fly(m, precision, nb, V, ldv, W, ldw, s);
    return;
  }
  if (precision == TRBL_FP64) run_hv<double>(m, nb, V, ldv, W, ldw, s);
  else run_hv<float>(m, nb, V, ldv, W, ldw, s);
  TRBL_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ basis indexing on the device
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

// mask[i] = 1 when basis state i has at most maxp nucleons in the states of `set`
__global__ void occupation_mask_kernel(RankArgs a, uint64_t set, int maxp, int64_t D, double* mask) {
  const int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (x >= D) return;
  int lo = 0, hi = a.nblocks - 1;
  while (lo < hi) {  // last block with offset <= x
    const int mid = (lo + hi + 1) >> 1;
    if (a.blk_off[mid] <= x) lo = mid;
    else hi = mid - 1;
  }
  const int64_t rel = x - a.blk_off[lo];
  const int dn = a.blk_dn[lo];
  const uint64_t pw = a.words[0][a.blk_p0[lo] + rel / dn];
  const uint64_t nw = a.words[1][a.blk_n0[lo] + rel % dn];
  mask[x] = (__popcll(pw & set) + __popcll(nw & set) <= maxp) ? 1.0 : 0.0;
}


void launch_rank(const Model& m, const uint64_t* pb, const uint64_t* nbits, int64_t n, int64_t* idx, hipStream_t s) {
  if (n <= 0) return;
  RankArgs a = rank_args(m);
  const int64_t nbk = (n + 255) / 256;
  hipLaunchKernelGGL(rank_kernel, dim3((unsigned)nbk), dim3(256), 0, s, a, pb, nbits, n, idx);
  TRBL_HIP(hipGetLastError());
}

void launch_occupation_mask(const Model& m, const int* orbit_set, int n_set, int maxp, double* mask, hipStream_t s) {
  uint64_t set = 0;
  for (int k = 0; k < n_set; k++) {
    TRBL_REQUIRE(orbit_set[k] >= 0 && orbit_set[k] < (int)m.orbits.size(), TRBL_E_INVALID, "orbit index out of range");
    for (int st = 0; st < m.ns; st++)
      if (m.st_orb[st] == orbit_set[k]) set |= 1ull << st;
  }
  RankArgs a = rank_args(m);
  const int64_t nbk = (m.dim + 255) / 256;
  hipLaunchKernelGGL(occupation_mask_kernel, dim3((unsigned)nbk), dim3(256), 0, s, a, set, maxp, m.dim, mask);
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
