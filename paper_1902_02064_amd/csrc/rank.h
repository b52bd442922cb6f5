// Device-side ranking of Slater determinants (App. A): the arguments shared by the basis
// indexing kernels (hv.hip) and the one-body jump generation (jumps.hip).
#pragma once
#include "internal.h"

namespace trbl {

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

__device__ inline uint64_t rev_bits(uint64_t w, int ns) { return __brevll(w) >> (64 - ns); }

// rank of word w inside its species sector, or -1
__device__ inline int species_rank(const RankArgs& a, int s, uint64_t w, int* sector) {
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


inline RankArgs rank_args(const Model& m) {
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

}  // namespace trbl
