// Gradient of sum_k w_k E_k with respect to the J-coupled two-body matrix elements
// and the single-particle energies. H is linear in its parameters, so by
// Hellmann-Feynman dE_k/dtheta = <psi_k| dH/dtheta |psi_k>; with
// H2 = sum_terms h_term O_term and h_term = sum_t c(term, t) V_t,
//   d(sum_k w_k E_k)/dV_t = sum_terms c(term, t) rho_term,
//   rho_term = sum_k w_k <psi_k| O_term |psi_k>   (two-body densities).
// The densities are accumulated on the device with the same enumeration as the
// block H.V (identical-particle operator entries with their m-scheme terms;
// proton x neutron one-body jumps for the pn terms); the contraction with the
// coefficients c(term, t) of the J -> m conversion is done on the host.
#include "dense.h"

namespace trbl {

struct GradArgs {
  const double* X;  // [D][n] eigenvectors
  int n;
  const double* w;  // [n] weights (device)
  int nblocks, ncl, tjmax;
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
  const int* nj_start;
  const int2* nj_pack;
  const int* h_off;
  const int* h_ncol;
  const int* pp_ptr;
  const int* pp_col;
  const int* pp_tptr;
  const int* pp_tid;
  const int8_t* pp_tsgn;
  const int* nn_ptr;
  const int* nn_col;
  const int* nn_tptr;
  const int* nn_tid;
  const int8_t* nn_tsgn;
  double* rho_pn_bins;  // h-table layout
  double* rho_pp;       // per pp term
  double* rho_nn;       // per nn term
  double* occ;          // [2][norb] single-particle occupation densities
  int norb, ns;
  uint64_t orbmask[16];
  const uint64_t* pwords;
  const uint64_t* nwords;
};

// weighted overlap sum_c w_c x[c] y[c]
__device__ __forceinline__ double wdot(const double* x, const double* y, const double* w, int n) {
  double s = 0.0;
  for (int c = 0; c < n; c++) s += w[c] * x[c] * y[c];
  return s;
}

// pn densities: one workgroup per (block, proton row), one thread per target n' (strided)
__global__ __launch_bounds__(256) void dens_pn_kernel(GradArgs a) {
  int b = 0;
  int64_t item = blockIdx.x, base = 0;
  for (; b < a.nblocks; b++) {
    if (item < base + a.blk_dp[b]) break;
    base += a.blk_dp[b];
  }
  if (b >= a.nblocks) return;
  const int pl = (int)(item - base);
  const int dn = a.blk_dn[b];
  const int64_t off = a.blk_off[b];
  const int gp = a.blk_p0[b] + pl, gn0 = a.blk_n0[b];
  const int ncl = a.ncl;
  for (int nt = threadIdx.x; nt < dn; nt += blockDim.x) {
    const double* xt = a.X + (off + (int64_t)pl * dn + nt) * a.n;
    for (int cls = 0; cls < ncl; cls++) {
      const int sb = a.src_blk[b * ncl + cls];
      if (sb < 0) continue;
      const int j0 = a.pj_start[gp * ncl + cls], j1 = a.pj_start[gp * ncl + cls + 1];
      if (j0 == j1) continue;
      const int cn = (2 * a.tjmax - cls / 2) * 2 + (cls & 1);
      const int* ns0 = a.nj_start + (int64_t)cn * (a.nn_total + 1) + gn0;
      const int k0 = ns0[nt], k1 = ns0[nt + 1];
      const int64_t soff = a.blk_off[sb];
      const int sdn = a.blk_dn[sb];
      double* bins = a.rho_pn_bins + a.h_off[cls];
      const int hn = a.h_ncol[cls];
      for (int j = j0; j < j1; j++) {
        const int pm = a.pj_meta[j];
        const double sj = (pm & 1) ? -1.0 : 1.0;
        const double* src = a.X + (soff + (int64_t)a.pj_idx[j] * sdn) * a.n;
        for (int k = k0; k < k1; k++) {
          const int2 e = a.nj_pack[k];
          const double sk = (e.y & 1) ? -1.0 : 1.0;
          const double d = wdot(xt, src + (int64_t)e.x * a.n, a.w, a.n);
          atomicAdd(bins + (pm >> 1) * hn + (e.y >> 1), sj * sk * d);
        }
      }
    }
  }
}

// pp densities: one workgroup per (block, proton row p'); each operator entry (p', p) gives
// d = sum_n w-overlap(X[p', n], X[p, n]) shared by its m-scheme terms.
__global__ __launch_bounds__(256) void dens_pp_kernel(GradArgs a) {
  __shared__ double red[256];
  int b = 0;
  int64_t item = blockIdx.x, base = 0;
  for (; b < a.nblocks; b++) {
    if (item < base + a.blk_dp[b]) break;
    base += a.blk_dp[b];
  }
  if (b >= a.nblocks) return;
  const int pl = (int)(item - base);
  const int dn = a.blk_dn[b];
  const int64_t off = a.blk_off[b];
  const int gp = a.blk_p0[b] + pl;
  for (int e = a.pp_ptr[gp]; e < a.pp_ptr[gp + 1]; e++) {
    if (a.pp_tptr[e] == a.pp_tptr[e + 1]) continue;  // single-particle energies only
    const int p = a.pp_col[e];
    double s = 0.0;
    for (int nt = threadIdx.x; nt < dn; nt += blockDim.x)
      s += wdot(a.X + (off + (int64_t)pl * dn + nt) * a.n, a.X + (off + (int64_t)p * dn + nt) * a.n, a.w, a.n);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
      if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0)
      for (int t = a.pp_tptr[e]; t < a.pp_tptr[e + 1]; t++) atomicAdd(a.rho_pp + a.pp_tid[t], a.pp_tsgn[t] * red[0]);
    __syncthreads();
  }
}

// nn densities: one workgroup per (block, neutron column n')
__global__ __launch_bounds__(256) void dens_nn_kernel(GradArgs a) {
  __shared__ double red[256];
  int b = 0;
  int64_t item = blockIdx.x, base = 0;
  for (; b < a.nblocks; b++) {
    if (item < base + a.blk_dn[b]) break;
    base += a.blk_dn[b];
  }
  if (b >= a.nblocks) return;
  const int nl = (int)(item - base);
  const int dn = a.blk_dn[b], dp = a.blk_dp[b];
  const int64_t off = a.blk_off[b];
  const int gn = a.blk_n0[b] + nl;
  for (int e = a.nn_ptr[gn]; e < a.nn_ptr[gn + 1]; e++) {
    if (a.nn_tptr[e] == a.nn_tptr[e + 1]) continue;
    const int n = a.nn_col[e];
    double s = 0.0;
    for (int p = threadIdx.x; p < dp; p += blockDim.x)
      s += wdot(a.X + (off + (int64_t)p * dn + nl) * a.n, a.X + (off + (int64_t)p * dn + n) * a.n, a.w, a.n);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
      if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0)
      for (int t = a.nn_tptr[e]; t < a.nn_tptr[e + 1]; t++) atomicAdd(a.rho_nn + a.nn_tid[t], a.nn_tsgn[t] * red[0]);
    __syncthreads();
  }
}

// occupation densities of every orbit, per species: sum_i (sum_k w_k X[i,k]^2) * N_a(i)
__global__ void dens_occ_kernel(GradArgs a, int64_t D) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= D) return;
  int lo = 0, hi = a.nblocks - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.blk_off[mid] <= i) lo = mid;
    else hi = mid - 1;
  }
  const int64_t rel = i - a.blk_off[lo];
  const int dn = a.blk_dn[lo];
  const uint64_t pw = a.pwords[a.blk_p0[lo] + rel / dn], nw = a.nwords[a.blk_n0[lo] + rel % dn];
  const double* x = a.X + i * a.n;
  const double u = wdot(x, x, a.w, a.n);
  for (int o = 0; o < a.norb; o++) {
    const int np = __popcll(pw & a.orbmask[o]), nn = __popcll(nw & a.orbmask[o]);
    if (np) atomicAdd(a.occ + o, u * np);
    if (nn) atomicAdd(a.occ + a.norb + o, u * nn);
  }
}

void tbme_gradient(const Model& m, int n_eig, const double* w, const double* X, double* grad_v, double* grad_spe,
                   hipStream_t s) {
  TRBL_REQUIRE(m.has_h, TRBL_E_STATE, "no Hamiltonian set");
  TRBL_REQUIRE(!m.fly, TRBL_E_INVALID,
               "gradient needs the stored identical-particle operator (not built for wide single-species spaces)");
  TRBL_REQUIRE((int)m.orbits.size() <= 16, TRBL_E_INVALID, "gradient supports at most 16 orbits");
  const DeviceTables& d = m.dt;
  const int norb = (int)m.orbits.size();
  const size_t npn = (size_t)m.h_off_host.back();
  DevBuf wd, bins, rpp, rnn, occ;
  wd.upload(std::vector<double>(w, w + n_eig));
  bins.alloc(std::max<size_t>(1, npn) * sizeof(double));
  rpp.alloc(std::max<size_t>(1, m.terms_pp.size()) * sizeof(double));
  rnn.alloc(std::max<size_t>(1, m.terms_nn.size()) * sizeof(double));
  occ.alloc(2 * norb * sizeof(double));
  TRBL_HIP(hipMemsetAsync(bins.p, 0, bins.bytes, s));
  TRBL_HIP(hipMemsetAsync(rpp.p, 0, rpp.bytes, s));
  TRBL_HIP(hipMemsetAsync(rnn.p, 0, rnn.bytes, s));
  TRBL_HIP(hipMemsetAsync(occ.p, 0, occ.bytes, s));
  GradArgs a{};
  a.X = X;
  a.n = n_eig;
  a.w = wd.as<double>();
  a.nblocks = (int)m.blocks.size();
  a.ncl = m.cl.nclass;
  a.tjmax = m.cl.tjmax;
  a.nn_total = m.nn_total;
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
  a.pp_tptr = d.pp_tptr.as<int>();
  a.pp_tid = d.pp_tid.as<int>();
  a.pp_tsgn = d.pp_tsgn.as<int8_t>();
  a.nn_ptr = d.nn_ptr.as<int>();
  a.nn_col = d.nn_col.as<int>();
  a.nn_tptr = d.nn_tptr.as<int>();
  a.nn_tid = d.nn_tid.as<int>();
  a.nn_tsgn = d.nn_tsgn.as<int8_t>();
  a.rho_pn_bins = bins.as<double>();
  a.rho_pp = rpp.as<double>();
  a.rho_nn = rnn.as<double>();
  a.occ = occ.as<double>();
  a.norb = norb;
  a.ns = m.ns;
  for (int o = 0; o < norb; o++) {
    uint64_t mask = 0;
    for (int q = 0; q < m.ns; q++)
      if (m.st_orb[q] == o) mask |= 1ull << q;
    a.orbmask[o] = mask;
  }
  a.pwords = d.pwords.as<uint64_t>();
  a.nwords = d.nwords.as<uint64_t>();
  int64_t rows = 0, cols = 0;
  for (const auto& b : m.blocks) {
    rows += b.dp;
    cols += b.dn;
  }
  hipLaunchKernelGGL(dens_pn_kernel, dim3((unsigned)rows), dim3(256), 0, s, a);
  hipLaunchKernelGGL(dens_pp_kernel, dim3((unsigned)rows), dim3(256), 0, s, a);
  hipLaunchKernelGGL(dens_nn_kernel, dim3((unsigned)cols), dim3(256), 0, s, a);
  hipLaunchKernelGGL(dens_occ_kernel, dim3((unsigned)((m.dim + 255) / 256)), dim3(256), 0, s, a, m.dim);
  TRBL_HIP(hipGetLastError());
  std::vector<double> hb(npn), hpp(m.terms_pp.size()), hnn(m.terms_nn.size()), ho(2 * norb);
  std::vector<int> hterm(npn);
  TRBL_HIP(hipMemcpyAsync(hb.data(), bins.p, npn * sizeof(double), hipMemcpyDeviceToHost, s));
  TRBL_HIP(hipMemcpyAsync(hpp.data(), rpp.p, hpp.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  TRBL_HIP(hipMemcpyAsync(hnn.data(), rnn.p, hnn.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  TRBL_HIP(hipMemcpyAsync(ho.data(), occ.p, ho.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  TRBL_HIP(hipMemcpyAsync(hterm.data(), d.h_term.p, npn * sizeof(int), hipMemcpyDeviceToHost, s));
  TRBL_HIP(hipStreamSynchronize(s));
  // contraction with the J -> m coefficients
  const size_t nv = m.tbme.size();
  for (size_t t = 0; t < nv; t++) grad_v[t] = 0.0;
  for (size_t k = 0; k < hpp.size(); k++)
    for (const auto& cv : m.coef_pp[k]) grad_v[cv.first] += cv.second * hpp[k];
  for (size_t k = 0; k < hnn.size(); k++)
    for (const auto& cv : m.coef_nn[k]) grad_v[cv.first] += cv.second * hnn[k];
  for (size_t q = 0; q < npn; q++) {
    if (hterm[q] < 0) continue;
    for (const auto& cv : m.coef_pn[hterm[q]]) grad_v[cv.first] += cv.second * hb[q];
  }
  if (grad_spe)
    for (int q = 0; q < 2 * norb; q++) grad_spe[q] = ho[q];
}

}  // namespace trbl
