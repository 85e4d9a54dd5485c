// gwl_sigma_from_coeffs_noalloc: the continued fraction and assembly of
// gwl_sigma_from_coeffs with every device buffer it needs (the coefficients
// staged from the host, the per-pair energies and signs, the frequencies in
// hartree and the per-pair Sigma before it is copied out) carved from one
// file-scope device array instead of the context's allocations.
//
// The array is a host-side stand-in in host code; its device address is
// taken once per device with hipGetSymbolAddress (gwl_setup binds the
// current device, the entry point binds a device it has not seen yet) and
// only that address is ever passed to a kernel or a copy.
#include <mutex>

#include "context.h"

namespace gwl {
namespace {

constexpr size_t kScratchBytes = (size_t)32 << 20;  // 32 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_bind_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (bound on first use).
void* scratch_for_current_device() {
  int dev = -1;
  GWL_HIP(hipGetDevice(&dev));
  GWL_CHECK(dev >= 0 && dev < kMaxDevices, GWL_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lk(g_bind_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    GWL_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    GWL_CHECK(p != nullptr, GWL_EDEVICE, "scratch array has no device address");
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

// e_n[p] = eps[n_idx[p]], eta_n[p] = +1 (occupied) / -1 (empty); omega to hartree.
__global__ void noalloc_prep_kernel(const int* __restrict__ n_idx, int npairs,
                                    const double* __restrict__ eps, int n_occ,
                                    double* __restrict__ e_n, double* __restrict__ eta_n,
                                    double* __restrict__ omega, int nomega) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < npairs) {
    const int n = n_idx[i];
    e_n[i] = eps[n];
    eta_n[i] = n < n_occ ? 1.0 : -1.0;
  }
  if (i < nomega) omega[i] = omega[i] / kHartreeEv;
}

// Carves 256-byte-aligned pieces off the scratch array, in order.
struct Carver {
  unsigned char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    T* p = reinterpret_cast<T*>(base + off);
    off += (count * sizeof(T) + 255) & ~(size_t)255;
    return p;
  }
};

size_t scratch_need(size_t P, size_t ld, size_t n_orb, size_t n_omega) {
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  return 2 * al(P * ld * 8) + al(P * 8) + 2 * al(P * 4) + 2 * al(P * 8) + al(n_orb * 8) +
         al(n_omega * 8) + al(P * n_omega * 16);
}

}  // namespace

void noalloc_bind_current_device() { (void)scratch_for_current_device(); }

}  // namespace gwl

using namespace gwl;

extern "C" gwl_status gwl_sigma_from_coeffs_noalloc(gwl_ctx* ctx, const int* n_idx,
                                                    int n_pairs, const double* alpha,
                                                    const double* beta, const double* p_norm2,
                                                    const int* lens, int ld,
                                                    const double* omega_ev, int n_omega,
                                                    double eta_ev, double* sigma_out) {
  try {
    GWL_CHECK(ctx != nullptr, GWL_EINVAL, "null context");
    GWL_CHECK(n_pairs >= 0 && n_omega >= 0, GWL_EINVAL, "negative count");
    if (n_pairs == 0 || n_omega == 0) {
      set_error("");
      return GWL_OK;
    }
    GWL_CHECK(n_idx && alpha && beta && p_norm2 && lens && omega_ev && sigma_out, GWL_EINVAL,
              "null pointer");
    GWL_CHECK(ld >= 1 && ld <= 4000, GWL_EINVAL, "ld must be in [1, 4000]");
    GWL_CHECK(std::isfinite(eta_ev) && eta_ev > 0, GWL_EINVAL, "eta must be > 0");
    GWL_CHECK(!ctx->lanczos_on_c(), GWL_EUNSUPPORTED,
              "the allocation-free variant covers the continued fraction only, not the "
              "quadrature option");
    for (int i = 0; i < n_pairs; ++i) {
      GWL_CHECK(n_idx[i] >= 0 && n_idx[i] < ctx->n_orb, GWL_EINVAL, "orbital out of range");
      GWL_CHECK(lens[i] >= 0 && lens[i] <= ld, GWL_EINVAL, "length out of range");
    }
    const size_t need = scratch_need(n_pairs, ld, ctx->n_orb, n_omega);
    GWL_CHECK(need <= kScratchBytes, GWL_EINVAL,
              "inputs need " + std::to_string(need) + " bytes of device scratch; the "
              "allocation-free variant holds " + std::to_string(kScratchBytes) +
              " (2 n_pairs ld + n_pairs (4 + 2 n_omega) + n_orb + n_omega doubles, each "
              "piece rounded up to 256 bytes)");
    int dev = -1;
    GWL_HIP(hipGetDevice(&dev));
    GWL_CHECK(dev == ctx->device, GWL_EINVAL, "the context's device is not the current one");
    Carver cv{static_cast<unsigned char*>(scratch_for_current_device())};
    const size_t P = n_pairs;
    double* ca = cv.take<double>(P * ld);
    double* cb = cv.take<double>(P * ld);
    double* n2 = cv.take<double>(P);
    int* ln = cv.take<int>(P);
    int* ni = cv.take<int>(P);
    double* en = cv.take<double>(P);
    double* et = cv.take<double>(P);
    double* eps = cv.take<double>(ctx->n_orb);
    double* om = cv.take<double>(n_omega);
    double* sig = cv.take<double>(P * n_omega * 2);
    hipStream_t st = ctx->stream;
    GWL_HIP(hipMemcpyAsync(ca, alpha, sizeof(double) * P * ld, hipMemcpyHostToDevice, st));
    GWL_HIP(hipMemcpyAsync(cb, beta, sizeof(double) * P * ld, hipMemcpyHostToDevice, st));
    GWL_HIP(hipMemcpyAsync(n2, p_norm2, sizeof(double) * P, hipMemcpyHostToDevice, st));
    GWL_HIP(hipMemcpyAsync(ln, lens, sizeof(int) * P, hipMemcpyHostToDevice, st));
    GWL_HIP(hipMemcpyAsync(ni, n_idx, sizeof(int) * P, hipMemcpyHostToDevice, st));
    GWL_HIP(hipMemcpyAsync(eps, ctx->eps_ha.data(), sizeof(double) * ctx->n_orb,
                           hipMemcpyHostToDevice, st));
    GWL_HIP(hipMemcpyAsync(om, omega_ev, sizeof(double) * n_omega, hipMemcpyHostToDevice, st));
    const int nprep = std::max(n_pairs, n_omega);
    noalloc_prep_kernel<<<ceil_div(nprep, 256), 256, 0, st>>>(ni, n_pairs, eps, ctx->nv, en,
                                                              et, om, n_omega);
    GWL_HIP(hipGetLastError());
    cfrac_sigma(n_pairs, ca, cb, ln, n2, ld, en, et, om, n_omega, eta_ev / kHartreeEv, ctx->tda,
                sig, st);
    GWL_HIP(hipMemcpyAsync(sigma_out, sig, sizeof(double) * P * n_omega * 2,
                           hipMemcpyDeviceToHost, st));
    GWL_HIP(hipStreamSynchronize(st));
    set_error("");
    return GWL_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::exception& e) {
    set_error(e.what());
    return GWL_EDEVICE;
  }
}
