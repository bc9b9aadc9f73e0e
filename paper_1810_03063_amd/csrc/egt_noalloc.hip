// egt_saddle_gap_noalloc: the saddle-point residual of Section 2 for callers
// that cannot allocate device memory (code under HIP graph capture, serving
// loops, harnesses that forbid hipMalloc).
//
// It runs the kernels of egt_saddle_gap -- the two products A y and A^T x,
// the two best-response passes over the treeplexes and the in-order sums of
// their root partials -- but its scratch (both products, both node-value
// buffers, the partial sums) is carved out of one file-scope device array of
// kNoallocScratchBytes, and the three results stay on the device.  The array
// is the library's: each device holds its own copy for the life of the
// process, at an address looked up once per device with
// hipGetSymbolAddress.  Every scratch element is written before it is read,
// so nothing is cleared between calls.  All calls on one device share the
// array: calls that overlap in time on one device race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "egt_internal.h"

namespace egt {

namespace {

constexpr size_t kNoallocScratchBytes = (size_t)160 << 20;  // 160 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};  // device address of `scratch`, per device

// Device address of this device's copy of the scratch array (looked up on the
// first call on the device, with that device current).
int scratch_for_device(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(EGT_EINVAL, "device ordinal out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(EGT_EDEVICE, "hipGetSymbolAddress(scratch) returned null");
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return EGT_OK;
}

// out = {gap, br_max_y, br_min_x} from the two trees' root partials, each
// tree's partials added in order from 0 (the order egt_saddle_gap uses), so
// the two entry points agree bit for bit.
__global__ __launch_bounds__(64) void gap_from_partials_kernel(const double* partial, int nb, double* out) {
  if (threadIdx.x != 0) return;
  double s[2];
  for (int k = 0; k < 2; ++k) {
    double v = 0.0;
    for (int b = 0; b < nb; ++b) v += partial[(size_t)k * nb + b];
    s[k] = v;
  }
  // gap = max_y x^T A y - min_x x^T A y = -BR_y(-A^T x) - BR_x(A y)
  out[0] = -s[1] - s[0];
  out[1] = -s[1];
  out[2] = s[0];
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

}  // namespace

// Scratch bytes a saddle gap of `g` takes (products, node values, partials).
size_t noalloc_gap_bytes(const egt_game* g) {
  size_t b = 0;
  for (int p = 0; p < 2; ++p) {
    b += align256(sizeof(double) * (size_t)g->hp[p].n_seq * g->ld);
    b += align256(sizeof(double) * (size_t)g->hp[p].n_nodes * g->ld);
  }
  b += align256(sizeof(double) * 2 * (size_t)kMaxPartials);
  return b;
}

size_t noalloc_scratch_limit() { return kNoallocScratchBytes; }

}  // namespace egt

using namespace egt;

extern "C" int egt_saddle_gap_noalloc(const egt_game* g, const double* x, const double* y, double* out3,
                                      hipStream_t stream) {
  if (!g || !x || !y || !out3) return fail(EGT_EINVAL, "null argument");
  const size_t need = noalloc_gap_bytes(g);
  if (need > kNoallocScratchBytes)
    return fail(EGT_EINVAL, "the game's saddle-gap scratch (" + std::to_string(need) +
                                " bytes) exceeds the fixed scratch of egt_saddle_gap_noalloc (" +
                                std::to_string(kNoallocScratchBytes) + " bytes)");
  int dev = -1;
  EGT_HIP(hipGetDevice(&dev));
  if (dev != g->device) return fail(EGT_EINVAL, "the game lives on another device than the current one");
  void* base = nullptr;
  const int rc = scratch_for_device(dev, &base);
  if (rc) return rc;
  unsigned char* cur = (unsigned char*)base;
  auto take = [&](size_t bytes) {
    void* r = cur;
    cur += align256(bytes);
    return r;
  };
  double* grad[2];
  double* V[2];
  for (int p = 0; p < 2; ++p) {
    grad[p] = (double*)take(sizeof(double) * (size_t)g->hp[p].n_seq * g->ld);
    V[p] = (double*)take(sizeof(double) * (size_t)g->hp[p].n_nodes * g->ld);
  }
  double* partial = (double*)take(sizeof(double) * 2 * (size_t)kMaxPartials);
  EGT_HIP(launch_gradient(g, 0, y, grad[0], stream));
  EGT_HIP(launch_gradient(g, 1, x, grad[1], stream));
  const Pass ps[2] = {{0, grad[0], 1.0, nullptr, 0.0, 0.0, V[0], nullptr},
                      {1, grad[1], -1.0, nullptr, 0.0, 0.0, V[1], nullptr}};
  EGT_HIP(launch_passes(g, ps, 2, nullptr, partial, stream));
  hipLaunchKernelGGL(gap_from_partials_kernel, dim3(1), dim3(64), 0, stream, partial, n_partials(g), out3);
  EGT_HIP(hipGetLastError());
  return EGT_OK;
}
