// Thick-restart block Lanczos driver (Alg. 4 and the restart equations of Sec. 3.4).
//
// Per block iteration k (all vector work on one HIP stream, all D-length data in HBM):
//   W := H V_k                           on-the-fly block H.V (hv.hip)
//   alpha_k := sym(V_k^T W)
//   W -= Q C1 ; C2 := Q^T W ; W -= Q C2   classical Gram-Schmidt twice against every
//                                         stored vector v_1 .. v_{k_x + p k}; C1 is the
//                                         column block k of T (exact Q^T H V_k), C2 computed
//   V_{k+1} beta_k := QR(W)               Cholesky QR, twice (beta = R2 R1, diag > 0)
//   T blocks (k,k) = alpha_k, (k+1,k) = beta_k, (k,k+1) = beta_k^T
//   diagonalise T^(k); rho_i = || beta_k U[last block rows, i] ||
// stop when rho_i <= tol * max|theta| for the n_eig lowest; restart when the next
// block would exceed l_m stored vectors:
//   v_k := sum_j v_j U_jk (k <= l_s),  V_1 := V_{k+1},  r := beta_k U[last block, 1:l_s],
//   T := [diag(theta_1..l_s) r^T ; r .],  k_x := l_s.
// Mixed precision: the stored vectors Q and H.V are FP32, and W is kept in the basis
// array's next block (FP32 storage; every projection, update, Gram matrix and the
// QR factors are computed in FP64); T and its eigenproblem are FP64; at the end an
// FP64 Rayleigh-Ritz step on the Ritz vectors refines the eigenvalues.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "dense.h"

namespace trbl {

namespace {

struct Events {
  hipEvent_t e[6];
  Events() {
    for (auto& x : e) TRBL_HIP(hipEventCreate(&x));
  }
  ~Events() {
    for (auto& x : e) (void)hipEventDestroy(x);
  }
  double ms(int a, int b) const {
    float t = 0.f;
    if (hipEventElapsedTime(&t, e[a], e[b]) != hipSuccess) return 0.0;
    return t * 1e-3;
  }
};

int64_t round4(int64_t x) { return (x + 3) / 4 * 4; }

}  // namespace

template <class TQ>
static int solve_t(const Model& m, const trbl_opts& o, double* evals, void* evecs, trbl_info* info) {
  constexpr bool mixed = sizeof(TQ) == 4;
  const int64_t D = m.dim;
  const int nb = o.nb, neig = o.n_eig, ls = o.l_s, lm = o.l_m;
  TRBL_REQUIRE(m.has_h, TRBL_E_STATE, "no Hamiltonian set");
  TRBL_REQUIRE(nb >= 1 && nb <= 64, TRBL_E_INVALID, "nb must be 1..64");
  TRBL_REQUIRE(neig >= 1 && neig <= ls, TRBL_E_INVALID, "need 1 <= n_eig <= l_s");
  TRBL_REQUIRE(ls + 2 * nb <= lm && (int64_t)lm <= D, TRBL_E_INVALID, "need l_s + 2 nb <= l_m <= D");
  // the projected matrix reaches l_m - nb rows before a restart (the next block is stored first)
  TRBL_REQUIRE(lm - nb <= EIG_NMAX, TRBL_E_INVALID,
               "l_m - nb above " + std::to_string(EIG_NMAX) + " (the device eigensolver's largest matrix)");
  TRBL_REQUIRE(o.tol > 0.0 && o.max_iter >= 1, TRBL_E_INVALID, "bad tol or max_iter");
  TRBL_REQUIRE(o.criterion == TRBL_CONV_RESIDUAL || o.criterion == TRBL_CONV_RITZ_CHANGE, TRBL_E_INVALID,
               "unknown convergence criterion");
  hipStream_t st = (hipStream_t)o.stream;
  // an FP32 residual cannot fall far below the FP32 rounding of H.V: floor the tolerance
  const double tol = mixed ? std::max(o.tol, 1e-5) : o.tol;
  const char* vb = std::getenv("TRBL_VERBOSE");
  const bool verbose = vb && vb[0] && vb[0] != '0';
  // testing aid (trbl.h): overwrite half of the first kept Ritz vector after the first restart,
  // a damaged basis that T cannot see, so that the check of the returned pairs must catch it
  const char* cr = std::getenv("TRBL_TEST_CORRUPT_RESTART");
  const bool corrupt_restart = cr && cr[0] == '1';
  const auto t_begin = std::chrono::steady_clock::now();

  const int64_t ldq = round4(lm);
  const int ldu = std::max(ls, neig);
  DevBuf Qb, Vkb, Wb, Tb, C1b, C2b, Rb, thb, Ub, rhob, stb;
  Qb.alloc((size_t)D * ldq * sizeof(TQ));
  Vkb.alloc((size_t)D * nb * sizeof(TQ));
  // FP64: the new block W is an FP64 work array. Mixed precision: H V_k lands in the basis
  // array's next column block (FP32), and the projections, the QR and the normalised block stay
  // there, so the basis can keep the memory of the FP64 block; an FP64 copy is made only on the
  // rare breakdown path.
  if (!mixed) Wb.alloc((size_t)D * nb * sizeof(double));
  auto w64 = [&]() {
    Wb.alloc((size_t)D * nb * sizeof(double));
    return Wb.as<double>();
  };
  Tb.alloc((size_t)lm * lm * sizeof(double));
  C1b.alloc((size_t)lm * nb * sizeof(double));
  C2b.alloc((size_t)lm * nb * sizeof(double));
  Rb.alloc((size_t)5 * nb * nb * sizeof(double));
  thb.alloc((size_t)lm * sizeof(double));
  Ub.alloc((size_t)lm * ldu * sizeof(double));
  rhob.alloc((size_t)std::max(neig, 64) * sizeof(double));
  stb.alloc(4 * sizeof(int));
  TQ* Q = Qb.as<TQ>();
  TQ* Vk = Vkb.as<TQ>();  // packed copy of the current block: H.V stages whole source rows
  double* W = Wb.as<double>();  // FP64 only (mixed: w64() on demand)
  double* T = Tb.as<double>();
  double* C1 = C1b.as<double>();
  double* C2 = C2b.as<double>();
  double* R1 = Rb.as<double>();
  double* R1i = R1 + nb * nb;
  double* R2 = R1i + nb * nb;
  double* R2i = R2 + nb * nb;
  double* beta = R2i + nb * nb;
  double* theta = thb.as<double>();
  double* U = Ub.as<double>();
  double* rho = rhob.as<double>();
  int* status = stb.as<int>();
  Scratch sc;
  EigWork ew;
  Events ev;

  // Column-by-column QR with replacement, for a block that Cholesky QR finds rank deficient
  // (breakdown / Krylov exhaustion): X = Wsrc (D x nb, FP64) is orthogonalised twice against
  // Q[:, :mprev] and the earlier new columns; a column whose remaining norm is <= 1e-10 of the
  // largest column norm is replaced by a random vector orthogonal to all of them, with a zero
  // diagonal entry of beta. Writes Q[:, mprev:mprev+nb] and beta (upper, W = V_new beta).
  int breakdowns = 0;
  DevBuf xb, cb, nrmb, rib;
  auto robust_qr = [&](const double* Wsrc, int mprev, uint64_t salt) {
    xb.alloc((size_t)D * sizeof(double));
    cb.alloc((size_t)(lm + nb) * sizeof(double));
    nrmb.alloc(sizeof(double));
    rib.alloc(sizeof(double));
    double* x = xb.as<double>();
    double* cdev = cb.as<double>();
    std::vector<double> bh((size_t)nb * nb, 0.0), ch(lm + nb);
    auto dot_xx = [&]() {
      double h;
      tn<double, double>(x, 1, 1, x, 1, 1, D, nrmb.as<double>(), sc, st);
      TRBL_HIP(hipMemcpyAsync(&h, nrmb.p, sizeof(double), hipMemcpyDeviceToHost, st));
      TRBL_HIP(hipStreamSynchronize(st));
      return std::sqrt(std::max(h, 0.0));
    };
    auto orth_against = [&](int mo, double* coef) {  // x -= Q[:, :mo] (Q[:, :mo]^T x), twice
      for (int pass = 0; pass < 2 && mo > 0; pass++) {
        tn<TQ, double>(Q, ldq, mo, x, 1, 1, D, cdev, sc, st);
        update<TQ, double>(Q, ldq, mo, cdev, x, 1, x, 1, 1, D, 0, nullptr, sc, st);
        if (coef) {
          TRBL_HIP(hipMemcpyAsync(ch.data(), cdev, mo * sizeof(double), hipMemcpyDeviceToHost, st));
          TRBL_HIP(hipStreamSynchronize(st));
          for (int i = 0; i < mo; i++) coef[i] += ch[i];
        }
      }
    };
    double wmax = 0.0;
    std::vector<double> wn(nb);
    for (int j = 0; j < nb; j++) {
      copy_cols<double, double>(Wsrc + j, nb, x, 1, D, 1, st);
      wn[j] = dot_xx();
      wmax = std::max(wmax, wn[j]);
    }
    for (int j = 0; j < nb; j++) {
      copy_cols<double, double>(Wsrc + j, nb, x, 1, D, 1, st);
      std::vector<double> coef(mprev + j, 0.0);
      orth_against(mprev + j, coef.data());
      for (int i = 0; i < j; i++) bh[(size_t)i * nb + j] = coef[mprev + i];
      double nr = dot_xx();
      if (!(nr > 1e-10 * wmax) || !(wmax > 0.0)) {
        random_block<double>(x, 1, D, 1, o.seed ^ (0x9E3779B97F4A7C15ull * (salt + 1 + j)), st);
        mask_rows<double>(x, 1, D, 1, o.mask, st);
        orth_against(mprev + j, nullptr);
        nr = dot_xx();
        TRBL_REQUIRE(nr > 0.0, TRBL_E_BREAKDOWN, "no vector left outside the Krylov basis");
        bh[(size_t)j * nb + j] = 0.0;
        breakdowns++;
      } else {
        bh[(size_t)j * nb + j] = nr;
      }
      const double inv = 1.0 / nr;
      TRBL_HIP(hipMemcpyAsync(rib.p, &inv, sizeof(double), hipMemcpyHostToDevice, st));
      apply_small<double, TQ>(x, 1, rib.as<double>(), Q + mprev + j, ldq, 1, D, false, sc, st);
    }
    TRBL_HIP(hipMemcpyAsync(beta, bh.data(), bh.size() * sizeof(double), hipMemcpyHostToDevice, st));
    TRBL_HIP(hipStreamSynchronize(st));
  };

  // H.V of the solve: with a mask on a single-species space generated per element, rows
  // outside the truncated space are not generated at all (they are zeroed afterwards anyway)
  auto apply_h = [&](int prec, int ncol, const void* V, int64_t ldv, void* Wo, int64_t ldw) {
    if (m.fly && o.mask) launch_fly(m, prec, ncol, V, ldv, Wo, ldw, st, o.mask);
    else launch_apply(m, prec, ncol, V, ldv, Wo, ldw, st);
  };

  // ---- start block V_1 (orthonormalised by Cholesky QR twice)
  if (o.v0)
    copy_cols<TQ, TQ>(static_cast<const TQ*>(o.v0), nb, Q, ldq, D, nb, st);
  else
    random_block<TQ>(Q, ldq, D, nb, o.seed, st);
  mask_rows<TQ>(Q, ldq, D, nb, o.mask, st);
  tn<TQ, TQ>(Q, ldq, nb, Q, ldq, nb, D, C1, sc, st);
  chol(C1, 1, nb, R1, R1i, nullptr, nullptr, status, st);
  if (mixed) {
    apply_small<TQ, TQ>(Q, ldq, R1i, Q, ldq, nb, D, true, sc, st);
    chol(sc.last_part, sc.last_G, nb, R2, R2i, nullptr, nullptr, status + 1, st);
    apply_small<TQ, TQ>(Q, ldq, R2i, Q, ldq, nb, D, false, sc, st);
  } else {
    apply_small<TQ, double>(Q, ldq, R1i, W, nb, nb, D, true, sc, st);
    chol(sc.last_part, sc.last_G, nb, R2, R2i, nullptr, nullptr, status + 1, st);
    apply_small<double, TQ>(W, nb, R2i, Q, ldq, nb, D, false, sc, st);
  }
  TRBL_HIP(hipMemsetAsync(T, 0, sizeof(double) * (size_t)lm * lm, st));
  int sth[4] = {0, 0, 0, 0};
  TRBL_HIP(hipMemcpyAsync(sth, status, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
  TRBL_HIP(hipStreamSynchronize(st));
  if (sth[0] || sth[1]) {  // rank-deficient start block: column-wise QR with replacement
    W = w64();
    if (o.v0) copy_cols<TQ, double>(static_cast<const TQ*>(o.v0), nb, W, nb, D, nb, st);
    else {
      random_block<TQ>(Q, ldq, D, nb, o.seed, st);
      copy_cols<TQ, double>(Q, ldq, W, nb, D, nb, st);
    }
    mask_rows<double>(W, nb, D, nb, o.mask, st);
    robust_qr(W, 0, 0);
  }

  int kx = 0, k = 0, it = 0, restarts = 0, mcur = 0;
  double hnorm = 0.0;
  std::vector<double> th(neig), rh(neig);
  double t_hv = 0, t_orth = 0, t_qr = 0, t_eig = 0, t_rst = 0;
  bool converged = false, last_orth = false;
  int next_check = 1, it_prev = 0;  // adaptive convergence-test schedule (check_every < 0)
  double r_prev = -1.0;
  std::vector<double> th_prev;  // Ritz values at the previous test (Ritz-change criterion)
  int nchk = 0;
  bool vk_current = false;  // Vk already holds the basis block at column c0 (stored there by the QR)
  for (it = 1; it <= o.max_iter; it++) {
    k++;
    const int c0 = kx + (k - 1) * nb;
    mcur = c0 + nb;
    if (!vk_current) copy_cols<TQ, TQ>(Q + c0, ldq, Vk, nb, D, nb, st);
    vk_current = false;
    TRBL_HIP(hipEventRecord(ev.e[0], st));
    // W := H V_k (mixed: in the basis array's next block, Wq)
    float* Wq = mixed ? reinterpret_cast<float*>(Q) + mcur : nullptr;
    if (mixed) {
      apply_h(TRBL_MIXED, nb, Vk, nb, Wq, ldq);
      mask_rows<float>(Wq, ldq, D, nb, o.mask, st);
    } else {
      apply_h(TRBL_FP64, nb, Vk, nb, W, nb);
      mask_rows<double>(W, nb, D, nb, o.mask, st);
    }
    TRBL_HIP(hipEventRecord(ev.e[1], st));
    // alpha_k = V_k^T W, then block classical Gram-Schmidt twice against all stored vectors.
    // The first pass takes its coefficients from T: in exact arithmetic Q^T H V_k is the
    // column block k of T (alpha_k, beta_{k-1}^T and, right after a restart, the coupling
    // to the Ritz vectors), so only those vectors are read; what that misses is of the
    // order of the rounding of a computed first pass, and the full second pass removes it.
    const int r_lo = k == 1 ? 0 : c0 - nb;
    if (mixed) {
      tn<float, float>((const float*)Q + c0, ldq, nb, Wq, ldq, nb, D, C1 + (size_t)c0 * nb, sc, st);
      t_alpha(T, lm, c0, nb, C1, st);
      t_column(T, lm, c0, r_lo, nb, C1, st);
      update<float, float, float>((const float*)Q + r_lo, ldq, mcur - r_lo, C1 + (size_t)r_lo * nb, Wq, ldq, Wq,
                                  ldq, nb, D, 0, nullptr, sc, st);
      tn<float, float>((const float*)Q, ldq, mcur, Wq, ldq, nb, D, C2, sc, st);
      update<float, float, float>((const float*)Q, ldq, mcur, C2, Wq, ldq, Wq, ldq, nb, D, 2, nullptr, sc, st);
    } else {
      tn<double, double>((const double*)Q + c0, ldq, nb, W, nb, nb, D, C1 + (size_t)c0 * nb, sc, st);
      t_alpha(T, lm, c0, nb, C1, st);
      t_column(T, lm, c0, r_lo, nb, C1, st);
      update<double, double>((const double*)Q + r_lo, ldq, mcur - r_lo, C1 + (size_t)r_lo * nb, W, nb, W, nb, nb, D,
                             0, nullptr, sc, st);
      tn<double, double>((const double*)Q, ldq, mcur, W, nb, nb, D, C2, sc, st);
      update<double, double>((const double*)Q, ldq, mcur, C2, W, nb, W, nb, nb, D, 2, nullptr, sc, st);
    }
    TRBL_HIP(hipEventRecord(ev.e[2], st));
    // V_{k+1} beta_k := QR(W): Cholesky QR twice
    chol(sc.last_part, sc.last_G, nb, R1, R1i, nullptr, nullptr, status, st);
    // the second factor's product also stores the new block packed into Vk, the H.V input of the
    // next iteration
    if (mixed) {
      apply_small<float, float>(Wq, ldq, R1i, Wq, ldq, nb, D, true, sc, st);
      chol(sc.last_part, sc.last_G, nb, R2, R2i, R1, beta, status + 1, st);
      apply_small<float, float>(Wq, ldq, R2i, Wq, ldq, nb, D, false, sc, st, reinterpret_cast<float*>(Vk), nb);
    } else {
      apply_small<double, double>(W, nb, R1i, W, nb, nb, D, true, sc, st);
      chol(sc.last_part, sc.last_G, nb, R2, R2i, R1, beta, status + 1, st);
      apply_small<double, TQ>(W, nb, R2i, Q + mcur, ldq, nb, D, false, sc, st, Vk, nb);
    }
    t_beta(T, lm, c0, mcur, nb, beta, st);
    TRBL_HIP(hipMemcpyAsync(sth, status, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
    TRBL_HIP(hipStreamSynchronize(st));
    if (sth[0] || sth[1]) {
      // breakdown: W was scaled in place; form it again (same arithmetic) and take the
      // column-wise QR with replacement (Vk already holds the rejected block: V_k again first)
      copy_cols<TQ, TQ>(Q + c0, ldq, Vk, nb, D, nb, st);
      if (mixed) {
        W = w64();
        apply_h(TRBL_MIXED, nb, Vk, nb, Wq, ldq);
        mask_rows<float>(Wq, ldq, D, nb, o.mask, st);
        tn<float, float>((const float*)Q, ldq, mcur, Wq, ldq, nb, D, C1, sc, st);
        update<float, float>((const float*)Q, ldq, mcur, C1, Wq, ldq, W, nb, nb, D, 1, C2, sc, st);
        update<float, double>((const float*)Q, ldq, mcur, C2, W, nb, W, nb, nb, D, 0, nullptr, sc, st);
      } else {
        apply_h(TRBL_FP64, nb, Vk, nb, W, nb);
        mask_rows<double>(W, nb, D, nb, o.mask, st);
        tn<double, double>((const double*)Q, ldq, mcur, W, nb, nb, D, C1, sc, st);
        update<double, double>((const double*)Q, ldq, mcur, C1, W, nb, W, nb, nb, D, 1, C2, sc, st);
        update<double, double>((const double*)Q, ldq, mcur, C2, W, nb, W, nb, nb, D, 0, nullptr, sc, st);
      }
      robust_qr(W, mcur, (uint64_t)it);
      t_beta(T, lm, c0, mcur, nb, beta, st);
      sth[0] = sth[1] = 0;
    } else {
      vk_current = true;
    }
    TRBL_HIP(hipEventRecord(ev.e[3], st));
    // diagonalise T^(k) (every check_every iterations and before every restart)
    const bool restart_next = mcur + 2 * nb > lm;
    const bool check_now = o.check_every < 0 ? it >= next_check : it % std::max(1, o.check_every) == 0;
    if (!restart_next && !check_now && it < o.max_iter) {
      TRBL_HIP(hipEventSynchronize(ev.e[3]));
      t_hv += ev.ms(0, 1);
      t_orth += ev.ms(1, 2);
      t_qr += ev.ms(2, 3);
      continue;
    }
    const int nvec = restart_next ? ls : std::min(neig, mcur);
    symeig(T, lm, mcur, nvec, theta, U, ldu, ew, restart_next, st);  // orthonormal U only where kept
    last_orth = restart_next;
    nchk = std::min(neig, mcur);
    resid(beta, nb, U, ldu, mcur, nchk, rho, st);
    TRBL_HIP(hipEventRecord(ev.e[4], st));
    TRBL_HIP(hipMemcpyAsync(th.data(), theta, nchk * sizeof(double), hipMemcpyDeviceToHost, st));
    double tmax = 0.0;
    TRBL_HIP(hipMemcpyAsync(&tmax, theta + mcur - 1, sizeof(double), hipMemcpyDeviceToHost, st));
    TRBL_HIP(hipMemcpyAsync(rh.data(), rho, nchk * sizeof(double), hipMemcpyDeviceToHost, st));
    TRBL_HIP(hipStreamSynchronize(st));
    t_hv += ev.ms(0, 1);
    t_orth += ev.ms(1, 2);
    t_qr += ev.ms(2, 3);
    t_eig += ev.ms(3, 4);
    hnorm = std::max(hnorm, std::max(std::fabs(th[0]), std::fabs(tmax)));
    bool ok = nchk == neig;
    int nconv_it = 0;
    if (o.criterion == TRBL_CONV_RITZ_CHANGE) {
      // Sec. 4.1: the wanted Ritz values stop moving (absolute change <= tol between tests)
      for (int i = 0; i < nchk; i++) {
        const bool still = (int)th_prev.size() == nchk && std::fabs(th[i] - th_prev[i]) <= o.tol;
        nconv_it += still;
        ok = ok && still;
      }
      th_prev.assign(th.begin(), th.begin() + nchk);
    } else {
      for (int i = 0; i < nchk; i++) nconv_it += rh[i] <= tol * hnorm;
      for (int i = 0; ok && i < nchk; i++) ok = rh[i] <= tol * hnorm;
    }
    if (verbose) {
      double rmax = 0.0;
      for (int i = 0; i < nchk; i++) rmax = std::max(rmax, rh[i]);
      std::fprintf(stderr, "trbl it %d m %d conv %d/%d rmax %.3e th0 %.10f | hv %.2f orth %.2f qr %.2f eig %.2f ms\n",
                   it, mcur, nconv_it, neig, rmax / std::max(hnorm, 1e-300), th[0], ev.ms(0, 1) * 1e3,
                   ev.ms(1, 2) * 1e3, ev.ms(2, 3) * 1e3, ev.ms(3, 4) * 1e3);
      std::fflush(stderr);
    }
    if (ok) {
      converged = true;
      break;
    }
    if (o.check_every < 0) {
      // adaptive schedule: extrapolate the decay of the worst residual ratio r = rho / (tol |H|)
      // seen since the previous test; test again a little before it is predicted to reach 1
      double r = nchk < neig ? 1e30 : 0.0;
      for (int i = 0; i < nchk; i++) r = std::max(r, rh[i] / (tol * hnorm));
      int gap = r <= 1e2 ? 1 : 1 << 30;  // no usable rate: every iteration when close, else at restarts
      if (r_prev > 0.0 && it > it_prev && r < r_prev) {
        const double rate = std::log(r_prev / r) / (it - it_prev);
        gap = std::max(1, (int)std::min(1e9, std::floor(0.75 * std::log(r) / rate)));
      }
      next_check = it + gap;
      r_prev = r;
      it_prev = it;
    }
    if (restart_next && it < o.max_iter) {
      TRBL_HIP(hipEventRecord(ev.e[4], st));
      // the packed block is free between iterations: the work buffer of restarts that keep more
      // than 208 vectors
      rowgemm<TQ, TQ>(Q, ldq, mcur, U, ldu, ls, Q, ldq, D, mcur, ls, nb, st, Vk, D * nb);
      t_restart(T, lm, lm, theta, ls, beta, nb, U, ldu, mcur, st);
      if (corrupt_restart && restarts == 0 && ls >= 2)  // testing aid: damage a kept Ritz vector
        copy_cols<TQ, TQ>(Q + 1, ldq, Q, ldq, D / 2, 1, st);
      TRBL_HIP(hipEventRecord(ev.e[5], st));
      TRBL_HIP(hipEventSynchronize(ev.e[5]));
      t_rst += ev.ms(4, 5);
      kx = ls;
      k = 0;
      restarts++;
      vk_current = false;  // the restart product may use Vk as its work buffer
    }
  }
  if (it > o.max_iter) it = o.max_iter;

  // ---- results: Ritz values and (optionally) Ritz vectors X = Q U[:, :n_eig]
  double t_refine = 0.0;
  std::vector<double> res(rh.begin(), rh.begin() + nchk);
  for (int i = 0; i < neig; i++) evals[i] = i < nchk ? th[i] : NAN;
  bool verified = true;
  if (!mixed || !o.refine) {
    // the convergence test may have used eigenvectors of T that were only normalised
    const int nv = std::min(neig, mcur);
    if (!last_orth) symeig(T, lm, mcur, nv, theta, U, ldu, ew, true, st);
    if (evecs) rowgemm<TQ, double>(Q, ldq, mcur, U, ldu, neig, static_cast<double*>(evecs), neig, D, -1, 0, 0, st);
    // The returned pairs are checked against H itself: ||H x - theta x|| in FP64 for every Ritz
    // pair, nb columns at a time (the W block holds H X, the packed block or a new one holds X
    // where the caller wants no vectors). rho from T equals it in exact arithmetic; a damaged
    // basis (which T cannot see) shows up here.
    // (mixed precision keeps no FP64 block during the iteration: an FP64 one of at most 8 GB here)
    const int w = mixed ? (int)std::max<int64_t>(1, std::min<int64_t>(nb, (int64_t)(8e9 / (16.0 * D)))) : nb;
    DevBuf Xown, Wfin;
    double* Wr = W;
    if (mixed) {
      Wfin.alloc((size_t)D * w * sizeof(double));
      Wr = Wfin.as<double>();
    }
    double* Xc = nullptr;
    if (!evecs) {
      if (sizeof(TQ) == 8) Xc = reinterpret_cast<double*>(Vk);
      else {
        Xown.alloc((size_t)D * w * sizeof(double));
        Xc = Xown.as<double>();
      }
    }
    DevBuf rs;
    rs.alloc((size_t)std::max(nv, 1) * 3 * sizeof(double));
    double* xhx = rs.as<double>() + nv;   // x^T H x
    double* xx = xhx + nv;                // x^T x
    for (int c = 0; c < nv; c += w) {
      const int cw = std::min(w, nv - c);
      const double* X;
      int64_t ldx;
      if (evecs) {
        X = static_cast<const double*>(evecs) + c;
        ldx = neig;
      } else {
        rowgemm<TQ, double>(Q, ldq, mcur, U + c, ldu, cw, Xc, cw, D, -1, 0, 0, st);
        X = Xc;
        ldx = cw;
      }
      apply_h(TRBL_FP64, cw, X, ldx, Wr, cw);
      mask_rows<double>(Wr, cw, D, cw, o.mask, st);
      resid_cols(Wr, cw, X, ldx, theta + c, cw, D, rs.as<double>() + c, sc, st);
      double* part = sc.partials((size_t)dot_cols_parts(D) * cw);
      dot_cols(Wr, cw, X, ldx, cw, D, part, xhx + c, st);
      dot_cols(X, ldx, X, ldx, cw, D, part, xx + c, st);
    }
    std::vector<double> tr(3 * (size_t)nv);
    TRBL_HIP(hipMemcpyAsync(tr.data(), rs.p, 3 * nv * sizeof(double), hipMemcpyDeviceToHost, st));
    TRBL_HIP(hipStreamSynchronize(st));
    // The scale is the largest Rayleigh quotient of the returned vectors with H itself (T's own
    // values would scale a damaged run's tolerance with the damage). Allowed: ten times the
    // tolerance (with the Ritz-change criterion, ten times the larger of that and T's estimate),
    // plus rounding.
    double scale = 0.0;
    for (int i = 0; i < nv; i++) scale = std::max(scale, std::fabs(tr[nv + i] / std::max(tr[2 * nv + i], 1e-300)));
    for (int i = 0; i < nv; i++) {
      tr[i] = std::sqrt(std::max(tr[i], 0.0));
      const double est = i < (int)res.size() ? res[i] : 0.0;
      const double base = o.criterion == TRBL_CONV_RITZ_CHANGE ? std::max(est, tol * scale) : tol * scale;
      if (!(tr[i] <= 10.0 * base + 1e-12 * scale)) verified = false;
    }
    tr.resize(nv);
    if (verbose && !verified) std::fprintf(stderr, "trbl: Ritz pairs fail the check against H\n");
    res.assign(tr.begin(), tr.end());
  } else {
    // FP64 Rayleigh-Ritz on span(X), X = Q U[:, :n_eig] stored in place in Q's first n_eig columns
    TRBL_HIP(hipEventRecord(ev.e[0], st));
    rowgemm<TQ, TQ>(Q, ldq, mcur, U, ldu, neig, Q, ldq, D, -1, 0, 0, st, Vk, D * nb);
    const int cw = (int)std::max<int64_t>(1, std::min<int64_t>(32, (int64_t)(8e9 / (16.0 * D))));
    DevBuf Xc, Hc, Sb, Gb, Mb, Lb, Yb, Yp, tmp, th2, st2;
    Xc.alloc((size_t)D * cw * sizeof(double));
    Hc.alloc((size_t)D * cw * sizeof(double));
    Sb.alloc((size_t)neig * neig * sizeof(double));
    Gb.alloc((size_t)neig * neig * sizeof(double));
    Mb.alloc((size_t)neig * neig * sizeof(double));
    Lb.alloc((size_t)neig * neig * sizeof(double));
    Yb.alloc((size_t)neig * neig * sizeof(double));
    Yp.alloc((size_t)neig * neig * sizeof(double));
    tmp.alloc((size_t)neig * cw * sizeof(double));
    th2.alloc((size_t)neig * sizeof(double));
    st2.alloc(sizeof(int));
    double* S = Sb.as<double>();
    double* G = Gb.as<double>();
    for (int c = 0; c < neig; c += cw) {
      const int w = std::min(cw, neig - c);
      copy_cols<TQ, double>(Q + c, ldq, Xc.as<double>(), w, D, w, st);
      apply_h(TRBL_FP64, w, Xc.as<double>(), w, Hc.as<double>(), w);
      mask_rows<double>(Hc.as<double>(), w, D, w, o.mask, st);
      tn<TQ, double>(Q, ldq, neig, Hc.as<double>(), w, w, D, tmp.as<double>(), sc, st);
      copy_cols<double, double>(tmp.as<double>(), w, S + c, neig, neig, w, st);
      tn<TQ, double>(Q, ldq, neig, Xc.as<double>(), w, w, D, tmp.as<double>(), sc, st);
      copy_cols<double, double>(tmp.as<double>(), w, G + c, neig, neig, w, st);
    }
    gen_reduce(S, G, neig, Mb.as<double>(), Lb.as<double>(), st2.as<int>(), st);
    symeig(Mb.as<double>(), neig, neig, neig, th2.as<double>(), Yp.as<double>(), neig, ew, false, st);
    gen_back(Lb.as<double>(), Yp.as<double>(), neig, neig, neig, Yb.as<double>(), neig, st);
    int gst = 0;
    TRBL_HIP(hipMemcpyAsync(evals, th2.as<double>(), neig * sizeof(double), hipMemcpyDeviceToHost, st));
    TRBL_HIP(hipMemcpyAsync(&gst, st2.as<int>(), sizeof(int), hipMemcpyDeviceToHost, st));
    // residual norms of the refined pairs in FP64, against H itself (the Ritz vectors formed
    // chunk by chunk where the caller wants none back)
    if (evecs)
      rowgemm<TQ, double>(Q, ldq, neig, Yb.as<double>(), neig, neig, static_cast<double*>(evecs), neig, D, -1, 0, 0,
                          st);
    DevBuf rs;
    rs.alloc((size_t)neig * sizeof(double));
    for (int c = 0; c < neig; c += cw) {
      const int w = std::min(std::min(cw, 64), neig - c);
      const double* X;
      int64_t ldx;
      if (evecs) {
        X = static_cast<const double*>(evecs) + c;
        ldx = neig;
      } else {
        rowgemm<TQ, double>(Q, ldq, neig, Yb.as<double>() + c, neig, w, Xc.as<double>(), w, D, -1, 0, 0, st);
        X = Xc.as<double>();
        ldx = w;
      }
      apply_h(TRBL_FP64, w, X, ldx, Hc.as<double>(), w);
      mask_rows<double>(Hc.as<double>(), w, D, w, o.mask, st);
      resid_cols(Hc.as<double>(), w, X, ldx, th2.as<double>() + c, w, D, rs.as<double>() + c, sc, st);
    }
    const std::vector<double> est = res;  // estimates from T for the unrefined pairs
    res.assign(neig, 0.0);
    TRBL_HIP(hipMemcpyAsync(res.data(), rs.as<double>(), neig * sizeof(double), hipMemcpyDeviceToHost, st));
    TRBL_HIP(hipStreamSynchronize(st));
    // scale: the refined eigenvalues are Rayleigh-Ritz values of H itself
    std::vector<double> th2h(neig);
    TRBL_HIP(hipMemcpy(th2h.data(), th2.p, neig * sizeof(double), hipMemcpyDeviceToHost));
    double scale = 0.0;
    for (double t : th2h) scale = std::max(scale, std::fabs(t));
    for (int i = 0; i < neig; i++) {
      res[i] = std::sqrt(std::max(res[i], 0.0));
      const double e = i < (int)est.size() ? est[i] : 0.0;
      const double base = o.criterion == TRBL_CONV_RITZ_CHANGE ? std::max(e, tol * scale) : tol * scale;
      if (!(res[i] <= 10.0 * base + 1e-12 * scale)) verified = false;
    }
    if (verbose && !verified) std::fprintf(stderr, "trbl: refined pairs fail the check against H\n");
    TRBL_HIP(hipEventRecord(ev.e[1], st));
    TRBL_HIP(hipStreamSynchronize(st));
    TRBL_REQUIRE(gst == 0, TRBL_E_BREAKDOWN, "refinement Gram matrix not positive definite");
    t_refine = ev.ms(0, 1);
  }
  TRBL_HIP(hipStreamSynchronize(st));
  if (info) {
    info->iterations = it;
    info->restarts = restarts;
    info->breakdowns = breakdowns;
    int nconv = 0;
    for (int i = 0; i < nchk; i++) nconv += rh[i] <= tol * hnorm;
    info->n_converged = nconv;
    info->t_hv = t_hv;
    info->t_orth = t_orth;
    info->t_qr = t_qr;
    info->t_eig = t_eig;
    info->t_restart = t_rst;
    info->t_refine = t_refine;
    info->t_total = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_begin).count();
    if (info->resid)
      for (int i = 0; i < neig; i++) info->resid[i] = i < (int)res.size() ? res[i] : NAN;
  }
  return converged && verified ? TRBL_OK : TRBL_NOT_CONVERGED;
}

int solve(const Model& m, const trbl_opts& o, double* evals, void* evecs, trbl_info* info) {
  if (o.precision == TRBL_FP64) return solve_t<double>(m, o, evals, evecs, info);
  TRBL_REQUIRE(o.precision == TRBL_MIXED, TRBL_E_INVALID, "bad precision");
  return solve_t<float>(m, o, evals, evecs, info);
}

}  // namespace trbl
