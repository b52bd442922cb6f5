// Host-side set-up of libtrbl: M-scheme basis (Sec. 2, App. A), J-coupled to
// m-scheme conversion of the interaction (Sec. 2), and the tables the H.V
// kernels read: identical-particle operator rows and one-body jumps (App. B).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <functional>
#include <map>
#include <tuple>

#include "internal.h"

namespace trbl {

// ------------------------------------------------------------------ Clebsch-Gordan
// Racah's closed formula in long double; arguments doubled. Factorials up to
// 34! are needed for 2j <= 31; long double keeps ~19 digits.
static long double lfact(int x2) {  // (x2/2)!
  static std::vector<long double> tab;
  if (tab.empty()) {
    tab.resize(200);
    tab[0] = 1.0L;
    for (int i = 1; i < 200; i++) tab[i] = tab[i - 1] * (long double)i;
  }
  return tab[x2 / 2];
}

double clebsch(int tj1, int tm1, int tj2, int tm2, int tJ, int tM) {
  if (tm1 + tm2 != tM) return 0.0;
  if (tJ < std::abs(tj1 - tj2) || tJ > tj1 + tj2 || ((tj1 + tj2 + tJ) & 1)) return 0.0;
  if (std::abs(tm1) > tj1 || std::abs(tm2) > tj2 || std::abs(tM) > tJ) return 0.0;
  if (((tj1 + tm1) & 1) || ((tj2 + tm2) & 1) || ((tJ + tM) & 1)) return 0.0;
  long double tri = lfact(tj1 + tj2 - tJ) * lfact(tj1 - tj2 + tJ) * lfact(-tj1 + tj2 + tJ) /
                    lfact(tj1 + tj2 + tJ + 2);
  long double pre = (long double)(tJ + 1) * tri * lfact(tj1 + tm1) * lfact(tj1 - tm1) * lfact(tj2 + tm2) *
                    lfact(tj2 - tm2) * lfact(tJ + tM) * lfact(tJ - tM);
  long double sum = 0.0L;
  for (int k = 0; 2 * k <= tj1 + tj2 + 2; k++) {
    int a[6] = {2 * k, tj1 + tj2 - tJ - 2 * k, tj1 - tm1 - 2 * k, tj2 + tm2 - 2 * k, tJ - tj2 + tm1 + 2 * k,
                tJ - tj1 - tm2 + 2 * k};
    bool ok = true;
    for (int q = 0; q < 6; q++) ok = ok && a[q] >= 0;
    if (!ok) continue;
    long double den = 1.0L;
    for (int q = 0; q < 6; q++) den *= lfact(a[q]);
    sum += ((k & 1) ? -1.0L : 1.0L) / den;
  }
  return (double)(sqrtl(pre) * sum);
}

// ------------------------------------------------------------------ basis
static int popc(uint64_t x) { return __builtin_popcountll(x); }
// the four low bits of x in reverse order
static int bitrev4(int x) { return ((x & 1) << 3) | ((x & 2) << 1) | ((x & 4) >> 1) | ((x & 8) >> 3); }

// Jordan-Wigner sign of an operator on state s of one species: (-1)^(occupied below s).
static int below_sign(uint64_t w, int s) {
  uint64_t low = s ? (w & ((1ull << s) - 1)) : 0ull;
  return (popc(low) & 1) ? -1 : 1;
}

// keep(2M, parity) selects the sectors that are stored (all when empty)
static void enumerate_species(const Model& m, Species& S, int npart,
                              const std::function<bool(int, int)>& keep = nullptr) {
  S.npart = npart;
  const int ns = m.ns;
  const int norb = (int)m.orbits.size();
  // count first to bound memory
  long double total = 1.0L;
  for (int i = 0; i < npart; i++) total = total * (ns - i) / (i + 1);
  TRBL_REQUIRE(total < 4.0e8L, TRBL_E_INVALID, "species space too large to enumerate");
  struct Item {
    uint64_t part, rev, word;
  };
  std::map<std::pair<int, int>, std::vector<Item>> sec;  // (2M, -parity) -> items
  auto visit = [&](uint64_t w) {
    int tm = 0, lsum = 0;
    int cnt[64] = {0};
    uint64_t rev = 0;
    for (uint64_t x = w; x; x &= x - 1) {
      int s = __builtin_ctzll(x);
      tm += m.st_tm[s];
      lsum += m.orbits[m.st_orb[s]].l;
      cnt[m.st_orb[s]]++;
      rev |= 1ull << (ns - 1 - s);
    }
    uint64_t part = 0;
    for (int o = 0; o < norb; o++) part = (part << 5) | (uint64_t)cnt[o];
    int par = (lsum & 1) ? -1 : 1;
    if (keep && !keep(tm, par)) return;
    sec[{tm, -par}].push_back({part, rev, w});
  };
  if (npart == 0) {
    visit(0);
  } else {
    uint64_t w = (npart == 64) ? ~0ull : ((1ull << npart) - 1);
    const uint64_t limit = (ns == 64) ? 0ull : (1ull << ns);
    while (true) {
      visit(w);
      // Gosper's hack: next larger word with the same popcount
      uint64_t c = w & (~w + 1), r = w + c;
      if (r == 0) break;
      uint64_t nw = (((r ^ w) >> 2) / c) | r;
      if (ns < 64 && nw >= limit) break;
      if (nw <= w) break;
      w = nw;
    }
  }
  S.words.clear();
  S.sectors.clear();
  S.sector_of.clear();
  S.part_key.clear();
  S.index.clear();
  for (auto& kv : sec) {
    auto& v = kv.second;
    std::sort(v.begin(), v.end(), [](const Item& a, const Item& b) {
      if (a.part != b.part) return a.part > b.part;  // partitions: descending lexicographic
      return a.rev > b.rev;                           // tuples: ascending lexicographic
    });
    SpeciesSector ss{kv.first.first, -kv.first.second, (int)S.words.size(), (int)v.size()};
    int id = (int)S.sectors.size();
    S.sectors.push_back(ss);
    for (auto& it : v) {
      S.index[it.word] = (int)S.words.size();
      S.words.push_back(it.word);
      S.part_key.push_back(it.part);
      S.sector_of.push_back(id);
    }
  }
}

void build_model(Model& m, const trbl_orbit* orbits, int n_orbits, int n_prot, int n_neut, int twoM, int parity) {
  TRBL_REQUIRE(orbits != nullptr && n_orbits > 0 && n_orbits <= 12, TRBL_E_INVALID, "need 1..12 orbits");
  TRBL_REQUIRE(parity >= -1 && parity <= 1, TRBL_E_INVALID, "parity must be -1, 0 or +1");
  m.orbits.assign(orbits, orbits + n_orbits);
  m.ns = 0;
  m.st_orb.clear();
  m.st_tm.clear();
  m.cl.tjmax = 0;
  for (int o = 0; o < n_orbits; o++) {
    const trbl_orbit& ob = orbits[o];
    TRBL_REQUIRE(ob.twoj > 0 && (ob.twoj & 1) && ob.l >= 0 && ob.n >= 0, TRBL_E_INVALID, "bad orbit");
    TRBL_REQUIRE(ob.twoj == 2 * ob.l + 1 || ob.twoj == 2 * ob.l - 1, TRBL_E_INVALID, "2j must be 2l +- 1");
    for (int tm = -ob.twoj; tm <= ob.twoj; tm += 2) {
      m.st_orb.push_back(o);
      m.st_tm.push_back(tm);
    }
    m.cl.tjmax = std::max(m.cl.tjmax, ob.twoj);
  }
  m.ns = (int)m.st_orb.size();
  TRBL_REQUIRE(m.ns <= 64, TRBL_E_TOO_MANY, "more than 64 m-states per species");
  TRBL_REQUIRE(n_prot >= 0 && n_prot <= m.ns && n_neut >= 0 && n_neut <= m.ns, TRBL_E_INVALID,
               "particle number out of range");
  m.cl.nclass = (2 * m.cl.tjmax + 1) * 2;
  m.n_prot = n_prot;
  m.n_neut = n_neut;
  m.twoM = twoM;
  m.parity = parity;
  // with one species empty only the sectors of the other that complete 2M and the parity are
  // stored (the others belong to no block and are reached by no operator of the space)
  auto keep_for = [&](int other) -> std::function<bool(int, int)> {
    if (other != 0) return nullptr;
    return [twoM, parity](int tm, int par) { return tm == twoM && (parity == 0 || par == parity); };
  };
  enumerate_species(m, m.sp[0], n_prot, keep_for(n_neut));
  enumerate_species(m, m.sp[1], n_neut, keep_for(n_prot));
  // blocks: 2M_p ascending, proton parity + first, neutron parity + first
  struct Key {
    int tmp, pp, pn, kp, kn;
  };
  std::vector<Key> keys;
  for (int kp = 0; kp < (int)m.sp[0].sectors.size(); kp++)
    for (int kn = 0; kn < (int)m.sp[1].sectors.size(); kn++) {
      const auto& a = m.sp[0].sectors[kp];
      const auto& b = m.sp[1].sectors[kn];
      if (a.twoM + b.twoM != twoM) continue;
      if (parity != 0 && a.par * b.par != parity) continue;
      keys.push_back({a.twoM, -a.par, -b.par, kp, kn});
    }
  std::sort(keys.begin(), keys.end(), [](const Key& x, const Key& y) {
    return std::tie(x.tmp, x.pp, x.pn) < std::tie(y.tmp, y.pp, y.pn);
  });
  m.blocks.clear();
  int64_t off = 0;
  m.max_dn = m.max_dp = 0;
  for (auto& k : keys) {
    BlockInfo b;
    b.psec = k.kp;
    b.nsec = k.kn;
    b.dp = m.sp[0].sectors[k.kp].size;
    b.dn = m.sp[1].sectors[k.kn].size;
    b.off = off;
    off += (int64_t)b.dp * b.dn;
    m.max_dn = std::max(m.max_dn, b.dn);
    m.max_dp = std::max(m.max_dp, b.dp);
    m.blocks.push_back(b);
  }
  m.dim = off;
  TRBL_REQUIRE(m.dim > 0, TRBL_E_EMPTY, "empty M-scheme space");
  m.np_total = (int64_t)m.sp[0].words.size();
  m.nn_total = (int64_t)m.sp[1].words.size();

  // device copies for rank / unrank and block layout
  const int nb = (int)m.blocks.size();
  std::vector<int> dp(nb), dn(nb), p0(nb), n0(nb);
  std::vector<int64_t> boff(nb + 1);
  for (int b = 0; b < nb; b++) {
    dp[b] = m.blocks[b].dp;
    dn[b] = m.blocks[b].dn;
    p0[b] = m.sp[0].sectors[m.blocks[b].psec].start;
    n0[b] = m.sp[1].sectors[m.blocks[b].nsec].start;
    boff[b] = m.blocks[b].off;
  }
  boff[nb] = m.dim;
  m.dt.blk_dp.upload(dp);
  m.dt.blk_dn.upload(dn);
  m.dt.blk_p0.upload(p0);
  m.dt.blk_n0.upload(n0);
  m.dt.blk_off.upload(boff);
  // block of (proton sector, neutron sector) for device ranking
  std::vector<int> bos(m.sp[0].sectors.size() * m.sp[1].sectors.size(), -1);
  for (int b = 0; b < nb; b++) bos[m.blocks[b].psec * m.sp[1].sectors.size() + m.blocks[b].nsec] = b;
  m.dt.blk_of_sec.upload(bos);
  for (int s = 0; s < 2; s++) {
    const Species& S = m.sp[s];
    std::vector<int> st, sz, tm, pr;
    for (auto& q : S.sectors) {
      st.push_back(q.start);
      sz.push_back(q.size);
      tm.push_back(q.twoM);
      pr.push_back(q.par);
    }
    (s == 0 ? m.dt.psec_tm : m.dt.nsec_tm).upload(tm);
    (s == 0 ? m.dt.psec_par : m.dt.nsec_par).upload(pr);
    (s == 0 ? m.dt.pwords : m.dt.nwords).upload(S.words);
    (s == 0 ? m.dt.ppart : m.dt.npart).upload(S.part_key);
    (s == 0 ? m.dt.psec_start : m.dt.nsec_start).upload(st);
    (s == 0 ? m.dt.psec_size : m.dt.nsec_size).upload(sz);
  }
  // source block of each (target block, proton jump class)
  const int ncl = m.cl.nclass;
  std::vector<int> src(nb * ncl, -1);
  std::map<std::tuple<int, int, int, int>, int> bidx;
  for (int b = 0; b < nb; b++) {
    const auto& a = m.sp[0].sectors[m.blocks[b].psec];
    const auto& c = m.sp[1].sectors[m.blocks[b].nsec];
    bidx[{a.twoM, a.par, c.twoM, c.par}] = b;
  }
  for (int b = 0; b < nb; b++) {
    const auto& a = m.sp[0].sectors[m.blocks[b].psec];
    const auto& c = m.sp[1].sectors[m.blocks[b].nsec];
    for (int cls = 0; cls < ncl; cls++) {
      int d2 = (cls / 2) * 2 - 2 * m.cl.tjmax;
      int flip = cls % 2;
      int fp = flip ? -1 : 1;
      auto it = bidx.find({a.twoM + d2, a.par * fp, c.twoM - d2, c.par * fp});
      if (it != bidx.end()) src[b * ncl + cls] = it->second;
    }
  }
  m.dt.src_blk.upload(src);
  m.src_blk_host = src;
  m.has_h = false;
  // single-species spaces too wide for the LDS-staged kernels (or any single-species space
  // when TRBL_FLY=1, a switch for testing) generate the identical-particle part on the fly
  m.fly = false;
  if ((n_prot == 0) != (n_neut == 0)) {
    m.fly_s = n_prot == 0 ? 1 : 0;
    int widest = 0;
    for (const auto& q : m.sp[m.fly_s].sectors) widest = std::max(widest, q.size);
    const char* env = std::getenv("TRBL_FLY");
    m.fly = widest > 2048 || (env && env[0] == '1');
  }
  if (m.fly) build_fly_basis(m);
}

// ------------------------------------------------------------------ interaction
namespace {

struct TermKey {
  int a, b, c, d;
  bool operator<(const TermKey& o) const { return std::tie(a, b, c, d) < std::tie(o.a, o.b, o.c, o.d); }
};

struct TermAcc {
  std::map<TermKey, int> id;
  std::vector<MTerm> terms;
  std::vector<std::vector<std::pair<int, double>>> coef;
  void add(int a, int b, int c, int d, double dh_dv, double v, int t) {
    auto it = id.find({a, b, c, d});
    int k;
    if (it == id.end()) {
      k = (int)terms.size();
      id[{a, b, c, d}] = k;
      terms.push_back({a, b, c, d, 0.0});
      coef.emplace_back();
    } else {
      k = it->second;
    }
    terms[k].h += dh_dv * v;
    auto& cv = coef[k];
    if (!cv.empty() && cv.back().first == t)
      cv.back().second += dh_dv;
    else
      cv.push_back({t, dh_dv});
  }
};

}  // namespace

void build_hamiltonian(Model& m, const double* spe_p, const double* spe_n, const trbl_tbme* v, int64_t n_v) {
  TRBL_REQUIRE(spe_p && spe_n, TRBL_E_INVALID, "single-particle energies required");
  TRBL_REQUIRE(n_v >= 0 && (n_v == 0 || v), TRBL_E_INVALID, "bad two-body list");
  const int norb = (int)m.orbits.size();
  const int ns = m.ns;
  m.spe[0].assign(spe_p, spe_p + norb);
  m.spe[1].assign(spe_n, spe_n + norb);
  m.tbme.assign(v, v + n_v);
  TermAcc acc[3];
  auto twoj = [&](int o) { return m.orbits[o].twoj; };
  for (int64_t t = 0; t < n_v; t++) {
    trbl_tbme e = v[t];
    TRBL_REQUIRE(e.channel >= 0 && e.channel <= 2, TRBL_E_INVALID, "channel must be 0, 1 or 2");
    TRBL_REQUIRE(e.a >= 0 && e.a < norb && e.b >= 0 && e.b < norb && e.c >= 0 && e.c < norb && e.d >= 0 &&
                     e.d < norb,
                 TRBL_E_INVALID, "orbit index out of range");
    TRBL_REQUIRE(e.twoJ >= 0 && !(e.twoJ & 1), TRBL_E_INVALID, "2J must be even and >= 0");
    auto tri = [&](int x, int y) { return e.twoJ >= std::abs(twoj(x) - twoj(y)) && e.twoJ <= twoj(x) + twoj(y); };
    TRBL_REQUIRE(tri(e.a, e.b) && tri(e.c, e.d), TRBL_E_INVALID, "J outside the triangle of a pair");
    TRBL_REQUIRE(((m.orbits[e.a].l + m.orbits[e.b].l + m.orbits[e.c].l + m.orbits[e.d].l) & 1) == 0,
                 TRBL_E_INVALID, "element breaks parity");
    const bool ident = e.channel != 2;
    double ph = 1.0;  // reordering phase: the canonical element is ph * v
    if (ident) {
      TRBL_REQUIRE(!(e.a == e.b && ((e.twoJ / 2) & 1)) && !(e.c == e.d && ((e.twoJ / 2) & 1)), TRBL_E_INVALID,
                   "identical nucleons in one j-shell couple to even J only");
      if (e.a > e.b) {
        std::swap(e.a, e.b);
        ph *= -((((twoj(e.a) + twoj(e.b) - e.twoJ) / 2) & 1) ? -1.0 : 1.0);
      }
      if (e.c > e.d) {
        std::swap(e.c, e.d);
        ph *= -((((twoj(e.c) + twoj(e.d) - e.twoJ) / 2) & 1) ? -1.0 : 1.0);
      }
    }
    // the pair of pair-states and its mirror
    int prs[2][4] = {{e.a, e.b, e.c, e.d}, {e.c, e.d, e.a, e.b}};
    int nmir = (e.a == e.c && e.b == e.d) ? 1 : 2;
    for (int q = 0; q < nmir; q++) {
      int A = prs[q][0], B = prs[q][1], C = prs[q][2], D = prs[q][3];
      double nab = (ident && A == B) ? std::sqrt(2.0) : 1.0;
      double ncd = (ident && C == D) ? std::sqrt(2.0) : 1.0;
      for (int s1 = 0; s1 < ns; s1++) {
        if (m.st_orb[s1] != A) continue;
        for (int s2 = 0; s2 < ns; s2++) {
          if (m.st_orb[s2] != B) continue;
          if (ident && s2 <= s1) continue;
          int tM = m.st_tm[s1] + m.st_tm[s2];
          double c1 = clebsch(twoj(A), m.st_tm[s1], twoj(B), m.st_tm[s2], e.twoJ, tM);
          if (c1 == 0.0) continue;
          for (int s3 = 0; s3 < ns; s3++) {
            if (m.st_orb[s3] != C) continue;
            for (int s4 = 0; s4 < ns; s4++) {
              if (m.st_orb[s4] != D) continue;
              if (ident && s4 <= s3) continue;
              if (m.st_tm[s3] + m.st_tm[s4] != tM) continue;
              double c2 = clebsch(twoj(C), m.st_tm[s3], twoj(D), m.st_tm[s4], e.twoJ, tM);
              if (c2 == 0.0) continue;
              acc[e.channel].add(s1, s2, s3, s4, ph * nab * ncd * c1 * c2, e.v, (int)t);
            }
          }
        }
      }
    }
  }
  m.terms_pp = acc[0].terms;
  m.terms_nn = acc[1].terms;
  m.terms_pn = acc[2].terms;
  m.coef_pp = acc[0].coef;
  m.coef_nn = acc[1].coef;
  m.coef_pn = acc[2].coef;

  // ---------------- identical-particle operator rows (App. B, first part), per species
  // Row g' of species s: <g'|H_ss|g> for every g reachable by a two-body jump, plus
  // the single-particle energies on the diagonal. Terms are grouped by creation pair
  // (a,b); the adjoint jump c+_c c+_d c_b c_a applied to g' gives g.
  if (m.fly) {  // identical-particle part generated per element; no pn part in this space
    build_fly_terms(m);
    build_fly_tiles(m);
    m.has_h = true;
    return;
  }
  // one-body operators c+_y c_x of each class (change of 2M and parity), numbered inside the
  // class; the same numbering for both species
  const Classes& cl = m.cl;
  const int ncl = cl.nclass;
  std::vector<std::vector<std::pair<int, int>>> pops(ncl);
  std::vector<int> op_idx(ns * ns), op_cls(ns * ns);
  for (int x = 0; x < ns; x++)
    for (int y = 0; y < ns; y++) {
      // jump from a determinant that removes x and adds y: its 2M changes by tm[y] - tm[x]
      const int d2 = m.st_tm[y] - m.st_tm[x];
      const int flip = (m.orbits[m.st_orb[x]].l + m.orbits[m.st_orb[y]].l) & 1;
      const int c = cl.cls(d2, flip);
      op_cls[x * ns + y] = c;
      op_idx[x * ns + y] = (int)pops[c].size();
      pops[c].push_back({x, y});
    }
  // the one-body jumps of each species are generated on the device; their counts per
  // (determinant, class) come first (the neutron lane order below needs them)
  JumpTables jt[2] = {JumpTables(m, 0), JumpTables(m, 1)};
  std::vector<int> jcount[2];
  for (int s = 0; s < 2; s++) {
    jt[s].set_ops(op_cls, op_idx);
    jcount[s] = jt[s].counts();
  }
  for (int s = 0; s < 2; s++) {
    const Species& S = m.sp[s];
    const std::vector<MTerm>& T = s == 0 ? m.terms_pp : m.terms_nn;
    std::vector<std::vector<int>> by_pair(ns * ns);
    for (int k = 0; k < (int)T.size(); k++) by_pair[T[k].a * ns + T[k].b].push_back(k);
    const std::vector<double>& e1 = m.spe[s];
    std::vector<int> ptr(1, 0), col;
    std::vector<double> val;
    std::vector<int> tptr(1, 0), tid;  // gradient: per entry, contributing (term, sign)
    std::vector<int8_t> tsg;
    std::vector<std::pair<int, std::pair<double, std::pair<int, int>>>> row;  // (g, (h, (term, sign)))
    for (int g = 0; g < (int)S.words.size(); g++) {
      uint64_t w = S.words[g];
      row.clear();
      double diag = 0.0;
      for (uint64_t x = w; x; x &= x - 1) diag += e1[m.st_orb[__builtin_ctzll(x)]];
      row.push_back({g, {diag, {-1, 0}}});
      for (uint64_t x = w; x; x &= x - 1) {
        int a = __builtin_ctzll(x);
        for (uint64_t y = x & (x - 1); y; y &= y - 1) {
          int b = __builtin_ctzll(y);
          for (int k : by_pair[a * ns + b]) {
            const MTerm& t = T[k];
            uint64_t r = w;
            int sg = below_sign(r, a);
            r &= ~(1ull << a);
            sg *= below_sign(r, b);
            r &= ~(1ull << b);
            if (r & (1ull << t.d)) continue;
            sg *= below_sign(r, t.d);
            r |= 1ull << t.d;
            if (r & (1ull << t.c)) continue;
            sg *= below_sign(r, t.c);
            r |= 1ull << t.c;
            auto it = S.index.find(r);
            if (it == S.index.end()) continue;
            row.push_back({it->second, {t.h * sg, {k, sg}}});
          }
        }
      }
      std::sort(row.begin(), row.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
      const int base = S.sectors[S.sector_of[g]].start;
      for (size_t i = 0; i < row.size();) {
        size_t j = i;
        double h = 0.0;
        while (j < row.size() && row[j].first == row[i].first) {
          h += row[j].second.first;
          if (row[j].second.second.first >= 0) {
            tid.push_back(row[j].second.second.first);
            tsg.push_back((int8_t)row[j].second.second.second);
          }
          j++;
        }
        col.push_back(row[i].first - base);
        val.push_back(h);
        tptr.push_back((int)tid.size());
        i = j;
      }
      ptr.push_back((int)col.size());
    }
    std::vector<float> val32(val.begin(), val.end());
    // Lane order of the rows kernel inside each neutron sector: SDs sorted by their number of
    // one-body jumps in each class (the class of no change first, then outwards), so that the
    // 64 targets of a wavefront have similar jump counts and few lanes idle while the longest
    // list of the wavefront is worked through. Protons keep the sector order.
    std::vector<int> lane_sd(S.words.size());
    for (size_t g = 0; g < S.words.size(); g++) lane_sd[g] = (int)(g - S.sectors[S.sector_of[g]].start);
    if (s == 1) {
      const int nc = m.cl.nclass;
      const std::vector<int>& cnt = jcount[1];
      std::vector<int> corder;  // classes by |change of 2M|, the unchanged class first
      for (int di = 0; di <= m.cl.tjmax * 2; di += 2)  // changes of 2M are even
        for (int f = 0; f < 2; f++)
          for (int sg = (di == 0 ? 1 : -1); sg <= 1; sg += 2) corder.push_back(m.cl.cls(sg * di, f));
      for (const auto& sec : S.sectors) {
        int* o = lane_sd.data() + sec.start;
        std::stable_sort(o, o + sec.size, [&](int a, int b) {
          for (int c : corder) {
            const int ca = cnt[(size_t)(sec.start + a) * nc + c], cb = cnt[(size_t)(sec.start + b) * nc + c];
            if (ca != cb) return ca > cb;
          }
          return false;
        });
      }
      m.dt.nlane.upload(lane_sd);
      m.nlane_pos.assign(S.words.size(), 0);
      for (const auto& sec : S.sectors)
        for (int r = 0; r < sec.size; r++) m.nlane_pos[sec.start + lane_sd[sec.start + r]] = r;
    }
    // sliced-ELL copy for the H.V kernels: slices of 64 consecutive lanes of one sector (one
    // wavefront of targets, in the lane order above), padded to the longest row of the slice,
    // entry k of lane l at base + k * 64 + l so the 64 lanes of a wavefront read 64 consecutive
    // entries.
    {
      std::vector<int> soff, sw, sec_slice0, ecol;
      std::vector<double> eval;
      for (const auto& sec : S.sectors) {
        sec_slice0.push_back((int)sw.size());
        for (int r0 = 0; r0 < sec.size; r0 += 64) {
          int w = 0;
          for (int r = r0; r < std::min(sec.size, r0 + 64); r++) {
            const int g = sec.start + lane_sd[sec.start + r];
            w = std::max(w, ptr[g + 1] - ptr[g]);
          }
          soff.push_back((int)ecol.size());
          sw.push_back(w);
          const size_t base = ecol.size();
          ecol.resize(base + (size_t)w * 64, 0);
          eval.resize(base + (size_t)w * 64, 0.0);
          for (int r = r0; r < std::min(sec.size, r0 + 64); r++) {
            const int g = sec.start + lane_sd[sec.start + r];
            // neutron rows in the bank order of the pn jump lists (the rows kernel gathers them
            // from the staged own row the same way)
            std::vector<int> ord(ptr[g + 1] - ptr[g]);
            for (size_t k = 0; k < ord.size(); k++) ord[k] = ptr[g] + (int)k;
            if (s == 1) {
              const int pref = bitrev4(r & 15);
              std::stable_sort(ord.begin(), ord.end(),
                               [&](int u, int v) { return bitrev4((col[u] ^ pref) & 15) < bitrev4((col[v] ^ pref) & 15); });
            }
            for (size_t k = 0; k < ord.size(); k++) {
              const size_t at = base + k * 64 + (r - r0);
              ecol[at] = col[ord[k]];
              eval[at] = val[ord[k]];
            }
          }
        }
      }
      std::vector<float> eval32(eval.begin(), eval.end());
      (s == 0 ? m.dt.pe_off : m.dt.ne_off).upload(soff);
      (s == 0 ? m.dt.pe_w : m.dt.ne_w).upload(sw);
      (s == 0 ? m.dt.pe_col : m.dt.ne_col).upload(ecol);
      (s == 0 ? m.dt.pe_v64 : m.dt.ne_v64).upload(eval);
      (s == 0 ? m.dt.pe_v32 : m.dt.ne_v32).upload(eval32);
      m.sec_slice0[s] = sec_slice0;
    }
    (s == 0 ? m.dt.pp_ptr : m.dt.nn_ptr).upload(ptr);
    (s == 0 ? m.dt.pp_col : m.dt.nn_col).upload(col);
    (s == 0 ? m.dt.pp_v64 : m.dt.nn_v64).upload(val);
    (s == 0 ? m.dt.pp_v32 : m.dt.nn_v32).upload(val32);
    (s == 0 ? m.dt.pp_tptr : m.dt.nn_tptr).upload(tptr);
    (s == 0 ? m.dt.pp_tid : m.dt.nn_tid).upload(tid);
    (s == 0 ? m.dt.pp_tsgn : m.dt.nn_tsgn).upload(tsg);
  }

  {
    std::vector<int> ps0, ns0;
    for (const auto& b : m.blocks) {
      ps0.push_back(m.sec_slice0[0][b.psec]);
      ns0.push_back(m.sec_slice0[1][b.nsec]);
    }
    m.dt.blk_pslice0.upload(ps0);
    m.dt.blk_nslice0.upload(ns0);
  }

  // ---------------- one-body jumps and the pn coefficient table (App. B, second part)
  // table h[cls][op_p][op_n] over proton class cls and neutron class conj(cls)
  std::vector<int> hoff(ncl + 1, 0), hncol(ncl, 0);
  for (int c = 0; c < ncl; c++) {
    hncol[c] = (int)pops[cl.conj(c)].size();
    hoff[c + 1] = hoff[c] + (int)pops[c].size() * hncol[c];
  }
  std::vector<double> h(hoff[ncl], 0.0);
  std::vector<int> hterm(hoff[ncl], -1);
  for (int k = 0; k < (int)m.terms_pn.size(); k++) {
    const MTerm& t = m.terms_pn[k];  // c+_a(p) c+_b(n) c_d(n) c_c(p): proton op (a,c), neutron op (b,d)
    const int c = op_cls[t.a * ns + t.c];
    const int cn = op_cls[t.b * ns + t.d];
    TRBL_REQUIRE(cn == cl.conj(c), TRBL_E_INVALID, "pn term breaks M or parity conservation");
    const int at = hoff[c] + op_idx[t.a * ns + t.c] * hncol[c] + op_idx[t.b * ns + t.d];
    h[at] += t.h;
    hterm[at] = k;
  }
  m.h_off_host = hoff;
  m.h_ncol_host = hncol;
  m.max_hncol = *std::max_element(hncol.begin(), hncol.end());
  std::vector<float> h32(h.begin(), h.end());
  m.dt.h_off.upload(hoff);
  m.dt.h_ncol.upload(hncol);
  m.dt.h64.upload(h);
  m.dt.h32.upload(h32);
  m.dt.h_term.upload(hterm);
  // Jump lists (device, jumps.hip): from each SD g' remove x in g', add y not in g' \ {x}
  // (y == x allowed). Proton side: per (SD, class), sorted by source index so equal source rows
  // are adjacent. Neutron side: class-major, so the lists of consecutive SDs in one class are
  // contiguous; each list has its number operators (source = the SD itself) first, then the
  // sources in the bank order of the SD's lane in the rows kernel (the kernel reads source row
  // n from LDS at n times the tile row size, so a source's low bits choose the part of a
  // 256-byte bank window its row lies in; the lane at position l prefers sources whose low four
  // bits match bitrev4(l mod 16), lowest bit first, so that at each step the lanes of a
  // wavefront spread over the window for every tile size at once).
  for (int s = 0; s < 2; s++) {
    const int64_t nsd = (int64_t)m.sp[s].words.size();
    const std::vector<int>& cnt = jcount[s];
    std::vector<int> start_gc(nsd * ncl + (s == 0 ? 1 : 0), 0);  // start of the (g, c) list, index g * ncl + c
    std::vector<int> start;                                      // the layout the kernels read
    int64_t total = 0;
    if (s == 0) {
      for (int64_t q = 0; q < nsd * ncl; q++) {
        start_gc[q] = (int)total;
        total += cnt[q];
      }
      start_gc[nsd * ncl] = (int)total;
      start = start_gc;
    } else {
      start.assign((int64_t)ncl * (nsd + 1), 0);
      for (int c = 0; c < ncl; c++) {
        for (int64_t g = 0; g < nsd; g++) {
          start[c * (nsd + 1) + g] = (int)total;
          start_gc[g * ncl + c] = (int)total;
          total += cnt[g * ncl + c];
        }
        start[c * (nsd + 1) + nsd] = (int)total;
      }
    }
    TRBL_REQUIRE(total < ((int64_t)1 << 31), TRBL_E_INVALID, "too many one-body jumps");
    std::vector<int> pref;
    if (s == 1) {
      pref.resize(nsd);
      for (int64_t g = 0; g < nsd; g++) pref[g] = bitrev4(m.nlane_pos[g] & 15);
    }
    DevBuf& jidx = s == 0 ? m.dt.pj_idx : m.dt.nj_idx;
    DevBuf& jmeta = s == 0 ? m.dt.pj_meta : m.dt.nj_meta;
    jt[s].fill(start_gc, total, pref, jidx, jmeta);
    (s == 0 ? m.dt.pj_start : m.dt.nj_start).upload(start);
    (s == 0 ? m.pj_count : m.nj_count) = (int)total;
    if (s == 1) {
      // neutron jumps packed in one word for the rows kernel: sign in bit 31, op index in
      // bits 16..30, source index inside its sector in bits 0..15
      int maxsec = 0, maxops = 0, mx = 0;
      for (const auto& sec : m.sp[1].sectors) maxsec = std::max(maxsec, sec.size);
      for (const auto& v : pops) maxops = std::max(maxops, (int)v.size());
      TRBL_REQUIRE(maxsec <= 65536 && maxops <= 32768, TRBL_E_INVALID,
                   "neutron sector or operator class too large for the packed jump lists");
      jt[1].pack(jidx, jmeta, total, m.dt.nj_pack, m.dt.nj32);
      for (int x : cnt) mx = std::max(mx, x);
      m.max_nj_class = mx;
    } else {
      // proton jump groups of every SD: runs of jumps of one class with one source row, class
      // by class, as (class, first jump, end jump, source row); per group the first group after
      // the run of its class
      const std::vector<int> ng = jt[0].group_counts(m.dt.pj_start, jidx);
      std::vector<int> gstart(nsd + 1, 0);
      int mg = 0;
      for (int64_t g = 0; g < nsd; g++) {
        int t = 0;
        for (int c = 0; c < ncl; c++) {
          t += ng[g * ncl + c];
          mg = std::max(mg, ng[g * ncl + c] * hncol[c]);
        }
        TRBL_REQUIRE((int64_t)gstart[g] + t < ((int64_t)1 << 31), TRBL_E_INVALID, "too many proton jump groups");
        gstart[g + 1] = gstart[g] + t;
      }
      m.max_hs_class = mg;
      m.dt.pg_start.upload(gstart);
      jt[0].group_fill(m.dt.pj_start, jidx, m.dt.pg_start, gstart[nsd], m.dt.pg_desc, m.dt.pg_cend);
    }
  }
  TRBL_HIP(hipDeviceSynchronize());
  build_pn_tiles(m);
  m.has_h = true;
}

}  // namespace trbl
