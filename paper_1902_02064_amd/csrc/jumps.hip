// One-body jump lists of each species, generated on the device (App. B: the proton-neutron
// part of H factorises into a proton jump c+_a c_c and a neutron jump c+_b c_d, and the jumps
// of every Slater determinant are listed once and reused by every block H.V).
//
// One thread per determinant g' of the species: for every occupied state x and every state y
// that is empty after removing x (y == x included: the number operators), the target word is
// ranked inside its sector by the device ranking of the basis, and the jump gets the
// Jordan-Wigner sign (-1)^(occupied states below x in g') * (-1)^(occupied states below y
// after the removal), both by popcount. Jumps are grouped by class (the change of 2M and of
// parity) and numbered inside the class by their (x, y) pair.
#include "rank.h"

namespace trbl {

namespace {

struct JumpArgs {
  RankArgs r;
  int s, ns, ncl, nsd;
  const uint64_t* words;  // the species' determinants in sector order (global index g')
  const int* ocls;        // class of the jump x -> y, [x * ns + y]
  const int* oidx;        // its number inside the class
};

__device__ inline int parity_below(uint64_t w, int x) { return __popcll(w & ((1ull << x) - 1)) & 1; }

// FILL = false: counts[g * ncl + c] = number of jumps of class c from g.
// FILL = true: the jumps written at cur[g * ncl + c] (their list starts, advanced here), then
// each list sorted in place: protons by source; neutrons own row first (the number operators),
// then by the bank-window preference of the determinant's lane (pref[g], the four low bits of
// the source compared lowest bit first), then by source. Sorting is stable, so equal keys keep
// the generation order (x ascending, then y ascending).
template <bool FILL>
__global__ void jump_kernel(JumpArgs a, int* counts, int* cur, const int* start, const int* pref, int* jidx,
                            int* jmeta) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= a.nsd) return;
  const uint64_t w = a.words[g];
  int* row = (FILL ? cur : counts) + (int64_t)g * a.ncl;
  if (!FILL)
    for (int c = 0; c < a.ncl; c++) row[c] = 0;
  for (uint64_t xx = w; xx; xx &= xx - 1) {
    const int x = __ffsll((long long)xx) - 1;
    const int sx = parity_below(w, x);
    const uint64_t r0 = w & ~(1ull << x);
    for (int y = 0; y < a.ns; y++) {
      if ((r0 >> y) & 1) continue;
      const uint64_t r = r0 | (1ull << y);
      int sec;
      const int local = species_rank(a.r, a.s, r, &sec);
      if (local < 0) continue;  // a sector that is not stored
      const int c = a.ocls[x * a.ns + y];
      if (!FILL) {
        row[c]++;
      } else {
        const int sign = sx ^ parity_below(r0, y);
        const int p = row[c]++;
        jidx[p] = local;
        jmeta[p] = (a.oidx[x * a.ns + y] << 1) | sign;
      }
    }
  }
  if (!FILL) return;
  int own_sec;
  const int own = species_rank(a.r, a.s, w, &own_sec);
  const int pf = pref ? pref[g] : 0;
  auto key = [&](int src) -> int64_t {
    if (a.s == 0) return src;
    if (src == own) return -1;
    const int d = (src ^ pf) & 15;
    const int k = ((d & 1) << 3) | ((d & 2) << 1) | ((d & 4) >> 1) | ((d & 8) >> 3);
    return ((int64_t)k << 32) | src;
  };
  for (int c = 0; c < a.ncl; c++) {
    const int b = start[(int64_t)g * a.ncl + c], e = row[c];
    for (int i = b + 1; i < e; i++) {  // insertion sort (lists of a few dozen)
      const int vi = jidx[i], mi = jmeta[i];
      const int64_t ki = key(vi);
      int j = i - 1;
      while (j >= b && key(jidx[j]) > ki) {
        jidx[j + 1] = jidx[j];
        jmeta[j + 1] = jmeta[j];
        j--;
      }
      jidx[j + 1] = vi;
      jmeta[j + 1] = mi;
    }
  }
}

// Proton jump groups: runs of one class with one source row. ngrp[g * ncl + c] counts them;
// the fill writes (class, first jump, end jump, source row) from gstart[g] and, per group, the
// first group after the run of its class (cend).
template <bool FILL>
__global__ void group_kernel(int nsd, int ncl, const int* start, const int* jidx, int* ngrp, const int* gstart,
                             int* gdesc, int* cend) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nsd) return;
  int q = FILL ? gstart[g] : 0;
  for (int c = 0; c < ncl; c++) {
    const int b = start[(int64_t)g * ncl + c], e = start[(int64_t)g * ncl + c + 1];
    const int q0 = q;
    for (int j = b; j < e;) {
      int je = j + 1;
      while (je < e && jidx[je] == jidx[j]) je++;
      if (FILL) {
        int* d = gdesc + 4 * (int64_t)q;
        d[0] = c;
        d[1] = j;
        d[2] = je;
        d[3] = jidx[j];
      }
      q++;
      j = je;
    }
    if (FILL)
      for (int t = q0; t < q; t++) cend[t] = q;
    else
      ngrp[(int64_t)g * ncl + c] = q - q0;
  }
}

// Neutron jumps packed for the kernels: (source, op << 1 | sign) pairs, and one word
// sign << 31 | op << 16 | source
__global__ void pack_kernel(int64_t n, const int* jidx, const int* jmeta, int2* pack, uint32_t* p32) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= n) return;
  const int i = jidx[q], m = jmeta[q];
  pack[q] = make_int2(i, m);
  p32[q] = ((uint32_t)(m & 1) << 31) | ((uint32_t)(m >> 1) << 16) | (uint32_t)i;
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

JumpTables::JumpTables(const Model& m, int s) : m_(m), s_(s) {
  ns_ = m.ns;
  ncl_ = m.cl.nclass;
  nsd_ = (int)m.sp[s].words.size();
}

void JumpTables::set_ops(const std::vector<int>& ocls, const std::vector<int>& oidx) {
  ocls_.upload(ocls);
  oidx_.upload(oidx);
}

std::vector<int> JumpTables::counts() {
  DevBuf cnt;
  cnt.alloc((size_t)nsd_ * ncl_ * sizeof(int));
  JumpArgs a{rank_args(m_), s_, ns_, ncl_, nsd_, (s_ == 0 ? m_.dt.pwords : m_.dt.nwords).as<uint64_t>(),
             ocls_.as<int>(), oidx_.as<int>()};
  if (nsd_ > 0)
    hipLaunchKernelGGL(jump_kernel<false>, dim3(blocks_for(nsd_)), dim3(256), 0, 0, a, cnt.as<int>(), nullptr,
                       nullptr, nullptr, nullptr, nullptr);
  TRBL_HIP(hipGetLastError());
  std::vector<int> h((size_t)nsd_ * ncl_);
  if (!h.empty()) TRBL_HIP(hipMemcpy(h.data(), cnt.p, h.size() * sizeof(int), hipMemcpyDeviceToHost));
  return h;
}

void JumpTables::fill(const std::vector<int>& start_gc, int64_t total, const std::vector<int>& pref, DevBuf& jidx,
                      DevBuf& jmeta) {
  DevBuf st, cur, pf;
  st.upload(start_gc);
  cur.upload(start_gc);
  if (!pref.empty()) pf.upload(pref);
  jidx.alloc((size_t)std::max<int64_t>(total, 1) * sizeof(int));
  jmeta.alloc((size_t)std::max<int64_t>(total, 1) * sizeof(int));
  JumpArgs a{rank_args(m_), s_, ns_, ncl_, nsd_, (s_ == 0 ? m_.dt.pwords : m_.dt.nwords).as<uint64_t>(),
             ocls_.as<int>(), oidx_.as<int>()};
  if (nsd_ > 0)
    hipLaunchKernelGGL(jump_kernel<true>, dim3(blocks_for(nsd_)), dim3(256), 0, 0, a, nullptr, cur.as<int>(),
                       st.as<int>(), pref.empty() ? nullptr : pf.as<int>(), jidx.as<int>(), jmeta.as<int>());
  TRBL_HIP(hipGetLastError());
  TRBL_HIP(hipDeviceSynchronize());
}

std::vector<int> JumpTables::group_counts(const DevBuf& start, const DevBuf& jidx) {
  DevBuf ng;
  ng.alloc((size_t)nsd_ * ncl_ * sizeof(int));
  if (nsd_ > 0)
    hipLaunchKernelGGL(group_kernel<false>, dim3(blocks_for(nsd_)), dim3(256), 0, 0, nsd_, ncl_, start.as<int>(),
                       jidx.as<int>(), ng.as<int>(), nullptr, nullptr, nullptr);
  TRBL_HIP(hipGetLastError());
  std::vector<int> h((size_t)nsd_ * ncl_);
  if (!h.empty()) TRBL_HIP(hipMemcpy(h.data(), ng.p, h.size() * sizeof(int), hipMemcpyDeviceToHost));
  return h;
}

void JumpTables::group_fill(const DevBuf& start, const DevBuf& jidx, const DevBuf& gstart, int ngroups, DevBuf& gdesc,
                            DevBuf& cend) {
  gdesc.alloc((size_t)std::max(ngroups, 1) * 4 * sizeof(int));
  cend.alloc((size_t)(ngroups + 1) * sizeof(int));
  const int tail = ngroups;  // the entry past the last group (read by nothing, kept defined)
  TRBL_HIP(hipMemcpy(cend.as<int>() + ngroups, &tail, sizeof(int), hipMemcpyHostToDevice));
  if (nsd_ > 0)
    hipLaunchKernelGGL(group_kernel<true>, dim3(blocks_for(nsd_)), dim3(256), 0, 0, nsd_, ncl_, start.as<int>(),
                       jidx.as<int>(), nullptr, gstart.as<int>(), gdesc.as<int>(), cend.as<int>());
  TRBL_HIP(hipGetLastError());
}

void JumpTables::pack(const DevBuf& jidx, const DevBuf& jmeta, int64_t n, DevBuf& pack, DevBuf& p32) {
  pack.alloc((size_t)std::max<int64_t>(n, 1) * sizeof(int2));
  p32.alloc((size_t)(n + 32) * sizeof(uint32_t));  // register loads read up to 32 past a list
  TRBL_HIP(hipMemset(p32.p, 0, (size_t)(n + 32) * sizeof(uint32_t)));
  if (n > 0)
    hipLaunchKernelGGL(pack_kernel, dim3(blocks_for(n)), dim3(256), 0, 0, n, jidx.as<int>(), jmeta.as<int>(),
                       pack.as<int2>(), p32.as<uint32_t>());
  TRBL_HIP(hipGetLastError());
}

}  // namespace trbl
