// Internal declarations shared by the host and device parts of libtrbl.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <memory>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/trbl.h"

namespace trbl {

// ---------------------------------------------------------------- errors
struct Error {
  int code;
  std::string msg;
};
void set_error(const std::string& msg);
#define TRBL_HIP(call)                                                                   \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      throw ::trbl::Error{TRBL_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)
#define TRBL_REQUIRE(cond, code, msg)                     \
  do {                                                    \
    if (!(cond)) throw ::trbl::Error{(code), (msg)};      \
  } while (0)

// Blocks of 256 lanes for a grid-stride loop over n elements. A dispatch describes its size in
// 32-bit work-item counts, so one lane per element would wrap beyond 2^32 elements (a D x 384
// block of a 1e8-dimensional space); the cap keeps every launch far below that.
inline unsigned elementwise_grid(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return (unsigned)(b < 1 ? 1 : b > (1 << 20) ? (1 << 20) : b);
}

// ---------------------------------------------------------------- device buffer
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  void alloc(size_t n) {
    if (n <= bytes && p) return;
    release();
    if (n == 0) n = 8;
    hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) {
      p = nullptr;
      throw Error{TRBL_E_NOMEM, "hipMalloc of " + std::to_string(n) + " bytes failed"};
    }
    bytes = n;
  }
  template <class T>
  void upload(const std::vector<T>& v) {
    alloc(v.size() * sizeof(T));
    if (!v.empty()) TRBL_HIP(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  }
  template <class T>
  T* as() const { return static_cast<T*>(p); }
};

// ---------------------------------------------------------------- model
struct SpeciesSector {
  int twoM, par;
  int start, size;  // global species index range
};

struct Species {
  int npart = 0;
  std::vector<uint64_t> words;                 // all SDs, sector by sector
  std::vector<int> sector_of;                  // global index -> sector id
  std::vector<SpeciesSector> sectors;          // ordered by (2M asc, parity + first)
  std::unordered_map<uint64_t, int> index;     // word -> global index
  std::vector<uint64_t> part_key;              // per SD: partition key (for device ranking)
};

struct BlockInfo {
  int psec, nsec;  // species sector ids
  int dp, dn;
  int64_t off;
};

// One-body jump classes: change of 2M (in steps of 2) and parity flip.
struct Classes {
  int tjmax = 0;   // largest 2j
  int nclass = 0;  // (2*tjmax+1) * 2
  int cls(int d2, int flip) const { return ((d2 + 2 * tjmax) / 2) * 2 + flip; }
  int conj(int c) const {  // class of the opposite-species jump: -d2, same flip
    int di = c / 2, f = c % 2;
    return (2 * tjmax - di) * 2 + f;
  }
};

struct DeviceTables {
  // blocks
  DevBuf blk_dp, blk_dn, blk_off, blk_p0, blk_n0, blk_item0, src_blk;
  // species words and sector info (for rank/unrank)
  DevBuf pwords, nwords, ppart, npart, psec_start, psec_size, nsec_start, nsec_size, blk_of_sec;
  DevBuf psec_tm, psec_par, nsec_tm, nsec_par;
  // jumps
  DevBuf pj_start, pj_idx, pj_meta, nj_start, nj_idx, nj_meta, nj_pack;  // nj_* class-major
  DevBuf pg_start, pg_desc;  // per proton SD: jump groups (class, first, end, source row) as int4
  DevBuf pg_cend;            // per jump group: first group after the run of its class
  DevBuf nj32;               // neutron jumps, class-major, packed: sign << 31 | op << 16 | source
  DevBuf nlane;              // per neutron SD slot (sector start + lane): the SD's index in its sector
  DevBuf h_off, h_ncol, h64, h32;
  DevBuf pp_ptr, pp_col, pp_v64, pp_v32, nn_ptr, nn_col, nn_v64, nn_v32;
  DevBuf pe_off, pe_w, pe_col, pe_v64, pe_v32, ne_off, ne_w, ne_col, ne_v64, ne_v32;  // sliced ELL
  DevBuf blk_pslice0, blk_nslice0;  // first ELL slice of each block's proton / neutron sector
  // gradient bins: per identical-particle operator entry / pn op pair, which m-scheme term
  DevBuf pp_term, nn_term;  // per CSR entry: list range into term lists
  DevBuf pp_tptr, pp_tid, pp_tsgn, nn_tptr, nn_tid, nn_tsgn;
  DevBuf h_term;            // per pn table entry: m-scheme pn term id (-1 if none)
  // one species only, generated on the fly (fly.hip): ranking tables and the two-body terms
  // grouped by creation pair
  DevBuf fly_base, fly_rank, fly_perm, fly_wint, fly_soff, fly_sstart, fly_pstart, fly_cd, fly_h64, fly_h32, fly_e64,
      fly_e32;
};

// Work decomposition of one block H.V (hv.hip), owned by the model. The rows kernel is
// launched once per bin of blocks with similar neutron-sector size, so that the LDS
// reservation and the workgroup width fit the sector.
struct HVBin {
  int nthr = 64, ntb = 256, nchunk = 1, rb_kb = 24, nblk = 0;  // width, its launch bound, chunks, LDS row KB
  int mp = 1;                                                    // targets per lane (1024-wide, 72 KB bins)
  int nr = 16;                                                   // neutron jumps per class held in registers
  int maxdn = 0;                                                 // widest target sector of the bin
  int64_t items = 0;
  DevBuf blocks, item0;  // block ids of the bin, first work item of each (nblk + 1)
};
struct HVPlan {
  int C = 1, ntile = 1, nchunk_c = 1, maxp_c = 1, nthr_c = 64;
  int Cc = 1, ntile_c = 1;  // columns kernel tile (narrower where the proton columns need it)
  int64_t cols_items = 0;
  size_t shm_c = 0;
  DevBuf citem0;
  std::vector<std::unique_ptr<HVBin>> bins;
};

// Proton-neutron part of H.V as dense pair blocks (pntile.hip). A proton determinant with one
// particle removed is a proton core K_p (the same for neutrons); every pn term moves one proton
// and one neutron, so it links the states K_p+x, K_n+u and K_p+y, K_n+v of exactly one core pair.
// With the pair states (x,u) of one total 2m listed once, the pn part is a sum over core pairs
// of the symmetric block H_M[(x,u)][(y,v)] restricted to the pairs outside the cores.
struct PNTiles {
  bool on = false;
  bool force = false;        // at every product width (TRBL_PN_TILES=2), not only the wide ones
  int S = 0;                 // contribution slots per basis state: n_prot * n_neut
  int nk = 0;                // pair blocks (2M of a pair from -2 tjmax to 2 tjmax)
  int nrect = 0;             // core-group rectangles (fixed core 2M and parity on both sides)
  int ncore[2] = {0, 0};
  int max_pairs = 0;         // widest pair block
  int tpb = 256;             // most core pairs of one work item
  int64_t items = 0;         // workgroups of one launch
  DevBuf cw[2], rk[2];       // core words; [core * ns + state]: position of state << 24 | local index of core + state, -1 inside
  DevBuf pr_off, pr_xu;      // pair blocks: x | u << 8
  DevBuf hb_off, hb, hb32;   // per pair block: D2 x D2 matrix (FP64, FP32), row = target pair
  DevBuf rect, rblk, item0;  // rectangles (pair block, rblk start), per rectangle and pair the target block
                             // (-1: none), work items (rectangle, proton core, first neutron core, count)
  DevBuf boff;               // block offsets as 32-bit integers
  hipStream_t side = nullptr;  // the columns kernel and the smaller own-row bins run here
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  PNTiles() = default;
  PNTiles(const PNTiles&) = delete;
  PNTiles& operator=(const PNTiles&) = delete;
  ~PNTiles() {
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
    if (side) (void)hipStreamDestroy(side);
  }
  DevBuf z;                  // slot buffer [S][D][16] of one 16-column tile (FP64, or FP32 in its first half)
};

// The identical-particle part of a single-species space as dense pair blocks (pntile.hip): cores
// of n - 2 nucleons, pairs (a < b) by (2M, parity), C(n, 2) slots per state.
struct FlyTiles {
  bool on = false;
  int S = 0, zw = 8, max_pairs = 0;
  int64_t items = 0;
  DevBuf cw;                         // cores, grouped by (2M, parity)
  DevBuf pr_off, pr_ab, hb_off, hb, hb32;
  DevBuf rect;                       // per rectangle: pair block, target sector
  DevBuf items_buf;                  // per work item: rectangle, first core, count, 0
  DevBuf z;                          // slot buffer [S][D][zw]
};

struct MTerm {  // m-scheme two-body term c+_a c+_b c_d c_c (species-local state indices)
  int a, b, c, d;
  double h;
};

struct Model {
  // space
  std::vector<trbl_orbit> orbits;
  int ns = 0;                      // m-states per species
  std::vector<int> st_orb, st_tm;  // per m-state: orbit, 2m
  int n_prot = 0, n_neut = 0, twoM = 0, parity = 0;
  Species sp[2];
  std::vector<BlockInfo> blocks;
  int64_t dim = 0;
  Classes cl;
  int device = 0;
  mutable std::unordered_map<int, std::unique_ptr<HVPlan>> hv_plans;  // key: nb * 16 + sizeof(T)
  // Hamiltonian
  bool has_h = false;
  std::vector<double> spe[2];
  std::vector<trbl_tbme> tbme;
  std::vector<MTerm> terms_pp, terms_nn, terms_pn;  // pn: a,c proton states; b,d neutron states
  // J-coupled element -> m-scheme term contributions (for the gradient contraction)
  std::vector<std::vector<std::pair<int, double>>> coef_pp, coef_nn, coef_pn;  // per term: (tbme idx, d h / d v)
  int64_t work_items_per_nb[2] = {0, 0};
  DeviceTables dt;
  // sizes for kernels
  int64_t np_total = 0, nn_total = 0;
  int pj_count = 0, nj_count = 0;
  int max_nj_class = 0;  // most neutron jumps of one SD in one class
  int max_hs_class = 0;  // most coefficient-table entries of one proton SD's jump groups of one class
  int max_hncol = 0;     // widest row of the pn coefficient table
  int max_dn = 0, max_dp = 0;
  std::vector<int> h_off_host, h_ncol_host;
  std::vector<int> src_blk_host;        // per (block, class): source block or -1
  std::vector<int> sec_slice0[2];       // per species sector: first sliced-ELL slice
  std::vector<int> nlane_pos;           // per neutron SD: its lane position in its sector
  // one species empty and the other's sector too wide for the LDS-staged kernels: the
  // identical-particle part is generated per element from the two-body terms (fly.hip)
  bool fly = false;
  int fly_s = 1;     // the occupied species
  int fly_half = 0;  // m-states in the low part of the two-level ranking
  mutable DevBuf fly_buf[2];  // V and W in the internal order (FP32, FP64)
  mutable FlyTiles flyt;      // its two-body part as dense pair blocks (when the slot buffer fits)
  mutable PNTiles pn;         // pn part as dense pair blocks (when its slot buffer fits)
};

// host helpers (model.cpp)
void build_model(Model& m, const trbl_orbit* orbits, int n_orbits, int n_prot, int n_neut, int twoM, int parity);
void build_hamiltonian(Model& m, const double* spe_p, const double* spe_n, const trbl_tbme* v, int64_t n_v);
// on-the-fly identical-particle H.V for single-species spaces (fly.hip)
void build_fly_basis(Model& m);
void build_fly_terms(Model& m);
void build_fly_tiles(Model& m);
// internal-order block product of a single-species space by pair blocks (Vint, Wint packed nb)
template <class T>
void launch_fly_tiles(const Model& m, int nb, const T* Vint, T* Wint, const double* mask, hipStream_t s);
// mask (optional, Table-1 order): rows with mask 0 are set to zero without being generated
void launch_fly(const Model& m, int precision, int nb, const void* V, int64_t ldv, void* W, int64_t ldw,
                hipStream_t s, const double* mask = nullptr);
double clebsch(int tj1, int tm1, int tj2, int tm2, int tJ, int tM);

// pn part by pair blocks (pntile.hip): tables built with the Hamiltonian; the product adds
// the pn part of H V to W (FP64, W already holding the identical-particle parts)
void build_pn_tiles(Model& m);
// (reduce false: the last 16-column tile stays in the slot buffer for the own-row kernel to sum)
template <class T>
void launch_pn_tiles(const Model& m, int nb, const T* V, int64_t ldv, T* W, int64_t ldw, hipStream_t s, bool reduce);

// device launchers (hv.hip)
void launch_apply(const Model& m, int precision, int nb, const void* V, int64_t ldv, void* W, int64_t ldw,
                  hipStream_t s);
// One-body jump lists of one species, generated on the device (jumps.hip): counts per
// (determinant, class) [g * ncl + c], the lists written at given starts and sorted, the proton
// jump groups, and the packed neutron forms.
class JumpTables {
 public:
  JumpTables(const Model& m, int s);
  void set_ops(const std::vector<int>& ocls, const std::vector<int>& oidx);
  std::vector<int> counts();
  void fill(const std::vector<int>& start_gc, int64_t total, const std::vector<int>& pref, DevBuf& jidx,
            DevBuf& jmeta);
  std::vector<int> group_counts(const DevBuf& start, const DevBuf& jidx);
  void group_fill(const DevBuf& start, const DevBuf& jidx, const DevBuf& gstart, int ngroups, DevBuf& gdesc,
                  DevBuf& cend);
  void pack(const DevBuf& jidx, const DevBuf& jmeta, int64_t n, DevBuf& pack, DevBuf& p32);

 private:
  const Model& m_;
  int s_, ns_ = 0, ncl_ = 0, nsd_ = 0;
  DevBuf ocls_, oidx_;
};
void launch_rank(const Model& m, const uint64_t* pb, const uint64_t* nb, int64_t n, int64_t* idx, hipStream_t s);
// build the block-product plans of the given column counts now (device tables of the work
// decomposition), so that later products of those widths allocate nothing
void prepare_hv_plans(const Model& m, int precision, const int* widths, int n);
bool has_hv_plan(const Model& m, int precision, int nb);
void launch_unrank(const Model& m, const int64_t* idx, int64_t n, uint64_t* pb, uint64_t* nb, hipStream_t s);
void launch_occupation_mask(const Model& m, const int* orbit_set, int n_set, int maxp, double* mask, hipStream_t s);

// solver (solver.cpp)
int solve(const Model& m, const trbl_opts& o, double* evals, void* evecs, trbl_info* info);
// gradient (grad.hip)
void tbme_gradient(const Model& m, int n_eig, const double* w, const double* X, double* grad_v,
                   double* grad_spe, hipStream_t s);

}  // namespace trbl

struct trbl_model {
  trbl::Model m;
};
