// C ABI of libtrbl (declared in include/trbl.h): argument checks, error
// capture, and dispatch to the host set-up, the H.V kernels and the solver.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "dense.h"

namespace trbl {
static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }
}  // namespace trbl

using trbl::Error;

template <class F>
static int guarded(F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    trbl::set_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    trbl::set_error("host allocation failed");
    return TRBL_E_NOMEM;
  } catch (const std::exception& e) {
    trbl::set_error(e.what());
    return TRBL_E_INVALID;
  } catch (...) {
    trbl::set_error("unknown error");
    return TRBL_E_INVALID;
  }
}

namespace trbl {
// the static scratch of trbl_expect_noalloc (64 MiB; see device_scratch below)
__device__ __align__(256) char scratch[(size_t)64 << 20];
}  // namespace trbl

namespace {

// The c-th output (0-based) of splitmix64 started from state `seed` (Steele, Lea and Flood,
// OOPSLA 2014, with Vigna's finaliser constants), so any draw can be made directly.
uint64_t splitmix64_at(uint64_t seed, uint64_t c) {
  uint64_t z = seed + (c + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
// uniform in (0, 1]: the top 53 bits plus one unit in the last place
double uniform01_at(uint64_t seed, uint64_t c) {
  return ((double)(splitmix64_at(seed, c) >> 11) + 1.0) * (1.0 / 9007199254740992.0);
}
// standard normal number k: Box-Muller (cosine branch) on uniforms 2k and 2k + 1
double normal_at(uint64_t seed, uint64_t k) {
  const double u1 = uniform01_at(seed, 2 * k), u2 = uniform01_at(seed, 2 * k + 1);
  return std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * 3.141592653589793 * u2);
}

// Scratch of trbl_expect_noalloc: one static array per device (the loader places a copy on each
// GPU the library runs on, held until the process ends). Host code never uses the array's name
// as an address: the device address comes from hipGetSymbolAddress, once per device.
constexpr size_t NOALLOC_BYTES = (size_t)64 << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex scratch_mu;
char* scratch_dev[NOALLOC_MAX_DEVICES] = {};

char* device_scratch() {
  int dev = 0;
  TRBL_HIP(hipGetDevice(&dev));
  TRBL_REQUIRE(dev >= 0 && dev < NOALLOC_MAX_DEVICES, TRBL_E_INVALID, "device index out of range");
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_dev[dev]) {
    void* p = nullptr;
    TRBL_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(trbl::scratch)));
    TRBL_REQUIRE(p != nullptr, TRBL_E_DEVICE, "no device address for the static scratch");
    scratch_dev[dev] = static_cast<char*>(p);
  }
  return scratch_dev[dev];
}

// column counts whose product plans trbl_set_hamiltonian prepares for trbl_expect_noalloc
constexpr int NOALLOC_WIDTHS[] = {1, 2, 4, 8, 16};

}  // namespace

extern "C" {

const char* trbl_last_error(void) { return trbl::g_last_error.c_str(); }

int trbl_random_tbme(const trbl_orbit* orbits, int n_orbits, uint64_t seed, double sigma, trbl_tbme* out,
                     int64_t capacity, int64_t* n_out) {
  return guarded([&] {
    TRBL_REQUIRE(orbits && n_orbits >= 1 && n_orbits <= 12 && n_out, TRBL_E_INVALID, "bad argument");
    TRBL_REQUIRE(capacity >= 0 && (out || capacity == 0), TRBL_E_INVALID, "bad output buffer");
    int tjmax = 0;
    for (int o = 0; o < n_orbits; o++) {
      TRBL_REQUIRE(orbits[o].twoj > 0 && (orbits[o].twoj & 1) && orbits[o].l >= 0, TRBL_E_INVALID, "bad orbit");
      tjmax = std::max(tjmax, orbits[o].twoj);
    }
    auto allows = [&](int ch, int a, int b, int tJ) {
      const int ja = orbits[a].twoj, jb = orbits[b].twoj;
      if (tJ < std::abs(ja - jb) || tJ > ja + jb) return false;
      return !(ch != 2 && a == b && ((tJ / 2) & 1));  // identical nucleons in one shell: even J
    };
    int64_t n = 0;
    uint64_t k = 0;
    std::vector<std::pair<int, int>> blk;
    for (int ch = 0; ch < 3; ch++)
      for (int tJ = 0; tJ <= 2 * tjmax; tJ += 2)
        for (int par = 1; par >= -1; par -= 2) {
          // pairs of the block: (a <= b) for pp and nn, every (a, b) for pn (a proton, b neutron)
          blk.clear();
          for (int a = 0; a < n_orbits; a++)
            for (int b = (ch == 2 ? 0 : a); b < n_orbits; b++)
              if ((((orbits[a].l + orbits[b].l) & 1) ? -1 : 1) == par && allows(ch, a, b, tJ)) blk.push_back({a, b});
          for (size_t i = 0; i < blk.size(); i++)
            for (size_t j = i; j < blk.size(); j++, k++, n++) {
              if (!out) continue;
              TRBL_REQUIRE(n < capacity, TRBL_E_INVALID, "output buffer too small");
              out[n] = trbl_tbme{ch, blk[i].first, blk[i].second, blk[j].first, blk[j].second, tJ,
                                 sigma * normal_at(seed, k)};
            }
        }
    *n_out = n;
    return TRBL_OK;
  });
}

int trbl_model_create(const trbl_orbit* orbits, int n_orbits, int n_prot, int n_neut, int twoM, int parity,
                      trbl_model** out) {
  return guarded([&] {
    TRBL_REQUIRE(out != nullptr, TRBL_E_INVALID, "out is NULL");
    *out = nullptr;
    auto* h = new trbl_model();
    try {
      TRBL_HIP(hipGetDevice(&h->m.device));
      trbl::build_model(h->m, orbits, n_orbits, n_prot, n_neut, twoM, parity);
    } catch (...) {
      delete h;
      throw;
    }
    *out = h;
    return TRBL_OK;
  });
}

void trbl_model_destroy(trbl_model* m) { delete m; }

int trbl_model_dim(const trbl_model* m, int64_t* dim) {
  return guarded([&] {
    TRBL_REQUIRE(m && dim, TRBL_E_INVALID, "NULL argument");
    *dim = m->m.dim;
    return TRBL_OK;
  });
}

int trbl_basis_unrank(const trbl_model* h, int64_t i, uint64_t* pbits, uint64_t* nbits) {
  return guarded([&] {
    TRBL_REQUIRE(h && pbits && nbits, TRBL_E_INVALID, "NULL argument");
    const trbl::Model& m = h->m;
    TRBL_REQUIRE(i >= 0 && i < m.dim, TRBL_E_INVALID, "index out of range");
    size_t lo = 0, hi = m.blocks.size() - 1;
    while (lo < hi) {
      size_t mid = (lo + hi + 1) / 2;
      if (m.blocks[mid].off <= i) lo = mid;
      else hi = mid - 1;
    }
    const auto& b = m.blocks[lo];
    int64_t rel = i - b.off;
    *pbits = m.sp[0].words[m.sp[0].sectors[b.psec].start + rel / b.dn];
    *nbits = m.sp[1].words[m.sp[1].sectors[b.nsec].start + rel % b.dn];
    return TRBL_OK;
  });
}

int trbl_basis_rank(const trbl_model* h, uint64_t pbits, uint64_t nbits, int64_t* i) {
  return guarded([&] {
    TRBL_REQUIRE(h && i, TRBL_E_INVALID, "NULL argument");
    const trbl::Model& m = h->m;
    *i = -1;
    auto ip = m.sp[0].index.find(pbits);
    auto in = m.sp[1].index.find(nbits);
    if (ip == m.sp[0].index.end() || in == m.sp[1].index.end()) return TRBL_OK;
    int kp = m.sp[0].sector_of[ip->second], kn = m.sp[1].sector_of[in->second];
    for (const auto& b : m.blocks)
      if (b.psec == kp && b.nsec == kn) {
        *i = b.off + (int64_t)(ip->second - m.sp[0].sectors[kp].start) * b.dn +
             (in->second - m.sp[1].sectors[kn].start);
        break;
      }
    return TRBL_OK;
  });
}

int trbl_basis_unrank_dev(const trbl_model* h, const int64_t* idx, int64_t n, uint64_t* pbits, uint64_t* nbits,
                          void* stream) {
  return guarded([&] {
    TRBL_REQUIRE(h && (n == 0 || (idx && pbits && nbits)) && n >= 0, TRBL_E_INVALID, "bad argument");
    trbl::launch_unrank(h->m, idx, n, pbits, nbits, (hipStream_t)stream);
    return TRBL_OK;
  });
}

int trbl_occupation_mask(const trbl_model* h, const int* orbit_set, int n_set, int max_particles, double* mask,
                         void* stream) {
  return guarded([&] {
    TRBL_REQUIRE(h && mask && n_set >= 0 && (n_set == 0 || orbit_set) && max_particles >= 0, TRBL_E_INVALID,
                 "bad argument");
    trbl::launch_occupation_mask(h->m, orbit_set, n_set, max_particles, mask, (hipStream_t)stream);
    return TRBL_OK;
  });
}

int trbl_basis_rank_dev(const trbl_model* h, const uint64_t* pbits, const uint64_t* nbits, int64_t n, int64_t* idx,
                        void* stream) {
  return guarded([&] {
    TRBL_REQUIRE(h && (n == 0 || (idx && pbits && nbits)) && n >= 0, TRBL_E_INVALID, "bad argument");
    trbl::launch_rank(h->m, pbits, nbits, n, idx, (hipStream_t)stream);
    return TRBL_OK;
  });
}

int trbl_set_hamiltonian(trbl_model* h, const double* spe_p, const double* spe_n, const trbl_tbme* tbme,
                         int64_t n_v) {
  return guarded([&] {
    TRBL_REQUIRE(h != nullptr, TRBL_E_INVALID, "NULL model");
    trbl::build_hamiltonian(h->m, spe_p, spe_n, tbme, n_v);
    trbl::prepare_hv_plans(h->m, TRBL_FP64, NOALLOC_WIDTHS, (int)(sizeof(NOALLOC_WIDTHS) / sizeof(int)));
    return TRBL_OK;
  });
}

int trbl_apply(const trbl_model* h, int precision, int nb, const void* V, void* W, void* stream) {
  return guarded([&] {
    TRBL_REQUIRE(h != nullptr, TRBL_E_INVALID, "NULL model");
    TRBL_REQUIRE(precision == TRBL_FP64 || precision == TRBL_MIXED, TRBL_E_INVALID, "bad precision");
    trbl::launch_apply(h->m, precision, nb, V, nb, W, nb, (hipStream_t)stream);
    return TRBL_OK;
  });
}

int trbl_expect(const trbl_model* h, int n, const void* X, double* out, void* stream) {
  return guarded([&] {
    TRBL_REQUIRE(h && X && out && n >= 1, TRBL_E_INVALID, "bad argument");
    const trbl::Model& m = h->m;
    hipStream_t s = (hipStream_t)stream;
    const int cw = 64;
    trbl::DevBuf Wb, Cb;
    Wb.alloc((size_t)m.dim * std::min(n, cw) * sizeof(double));
    Cb.alloc((size_t)cw * cw * sizeof(double));
    trbl::Scratch sc;
    std::vector<double> ch((size_t)cw * cw);
    const double* Xd = static_cast<const double*>(X);
    for (int c0 = 0; c0 < n; c0 += cw) {
      const int w = std::min(cw, n - c0);
      trbl::launch_apply(m, TRBL_FP64, w, Xd + c0, n, Wb.p, w, s);
      trbl::tn<double, double>(Xd + c0, n, w, Wb.as<double>(), w, w, m.dim, Cb.as<double>(), sc, s);
      TRBL_HIP(hipMemcpyAsync(ch.data(), Cb.p, (size_t)w * w * sizeof(double), hipMemcpyDeviceToHost, s));
      TRBL_HIP(hipStreamSynchronize(s));
      for (int j = 0; j < w; j++) out[c0 + j] = ch[(size_t)j * w + j];
    }
    return TRBL_OK;
  });
}

int trbl_expect_noalloc(const trbl_model* h, int n, const void* X, double* out, void* stream) {
  return guarded([&] {
    TRBL_REQUIRE(h && X && out && n >= 1, TRBL_E_INVALID, "bad argument");
    const trbl::Model& m = h->m;
    TRBL_REQUIRE(m.has_h, TRBL_E_STATE, "no Hamiltonian set");
    TRBL_REQUIRE(!m.fly, TRBL_E_INVALID, "single-species spaces generated per element keep work blocks; use trbl_expect");
    hipStream_t s = (hipStream_t)stream;
    const int64_t D = m.dim;
    static_assert(sizeof(trbl::scratch) == NOALLOC_BYTES, "scratch size");
    const size_t part_bytes = (size_t)trbl::dot_cols_parts(D) * 16 * sizeof(double);
    auto hx_bytes = [&](int w) { return ((size_t)D * w * sizeof(double) + 255) / 256 * 256; };
    // widest power-of-two chunk whose H X block fits the scratch beside the partial sums
    int w = 16;
    while (w > 1 && hx_bytes(w) + part_bytes > NOALLOC_BYTES) w >>= 1;
    TRBL_REQUIRE(hx_bytes(1) + part_bytes <= NOALLOC_BYTES, TRBL_E_INVALID,
                 "dimension too large for the " + std::to_string(NOALLOC_BYTES >> 20) + " MiB static scratch");
    char* sc = device_scratch();
    double* HX = reinterpret_cast<double*>(sc);
    double* part = reinterpret_cast<double*>(sc + hx_bytes(w));
    const double* Xd = static_cast<const double*>(X);
    for (int c0 = 0; c0 < n;) {
      int cw = w;
      while (cw > n - c0) cw >>= 1;  // the remainder in power-of-two pieces: plans exist for those
      TRBL_REQUIRE(trbl::has_hv_plan(m, TRBL_FP64, cw), TRBL_E_STATE, "product plan missing");
      trbl::launch_apply(m, TRBL_FP64, cw, Xd + c0, n, HX, cw, s);
      trbl::dot_cols(HX, cw, Xd + c0, n, cw, D, part, out + c0, s);
      c0 += cw;
    }
    return TRBL_OK;
  });
}

int trbl_solve(const trbl_model* h, const trbl_opts* opts, double* evals, void* evecs, trbl_info* info) {
  return guarded([&] {
    TRBL_REQUIRE(h && opts && evals, TRBL_E_INVALID, "NULL argument");
    return trbl::solve(h->m, *opts, evals, evecs, info);
  });
}

int trbl_tbme_grad(const trbl_model* h, const trbl_opts* opts, int n_eig, const double* w, const void* evecs,
                   double* grad_v, double* grad_spe) {
  return guarded([&] {
    TRBL_REQUIRE(h && w && grad_v && n_eig > 0, TRBL_E_INVALID, "bad argument");
    const trbl::Model& m = h->m;
    TRBL_REQUIRE(m.has_h, TRBL_E_STATE, "no Hamiltonian set");
    hipStream_t s = opts ? (hipStream_t)opts->stream : nullptr;
    trbl::DevBuf own;
    const double* X = static_cast<const double*>(evecs);
    if (!X) {
      TRBL_REQUIRE(opts != nullptr, TRBL_E_INVALID, "opts needed to recompute eigenvectors");
      TRBL_REQUIRE(opts->n_eig >= n_eig, TRBL_E_INVALID, "opts.n_eig smaller than n_eig");
      own.alloc((size_t)m.dim * opts->n_eig * sizeof(double));
      std::vector<double> ev(opts->n_eig);
      int rc = trbl::solve(m, *opts, ev.data(), own.p, nullptr);
      TRBL_REQUIRE(rc == TRBL_OK, rc < 0 ? rc : TRBL_E_BREAKDOWN, "eigenvector recomputation did not converge");
      // keep the n_eig lowest columns: [D][opts.n_eig] -> strided use below
      if (opts->n_eig != n_eig) {
        trbl::DevBuf tight;
        tight.alloc((size_t)m.dim * n_eig * sizeof(double));
        TRBL_HIP(hipMemcpy2DAsync(tight.p, n_eig * sizeof(double), own.p, opts->n_eig * sizeof(double),
                                  n_eig * sizeof(double), (size_t)m.dim, hipMemcpyDeviceToDevice, s));
        TRBL_HIP(hipStreamSynchronize(s));
        std::swap(own.p, tight.p);
        std::swap(own.bytes, tight.bytes);
      }
      X = own.as<double>();
    }
    trbl::tbme_gradient(m, n_eig, w, X, grad_v, grad_spe, s);
    return TRBL_OK;
  });
}

}  // extern "C"
