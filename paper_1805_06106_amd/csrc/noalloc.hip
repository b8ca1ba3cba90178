// gq_points_near_noalloc: the proximity query of gq_points_near with every device buffer
// taken from a fixed scratch array instead of hipMalloc, for callers that cannot allocate
// device memory.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/gigaqbx.h"
#include "kernels.hpp"
#include "query.hpp"

constexpr size_t kScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

#define NA_HIP(call)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return gq::set_error(GQ_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// The scratch: one copy per GPU, held until the process ends.  On the host `scratch` is a
// stand-in, not a device address: host code never passes it to a kernel or a copy, and
// uses the address that scratch_base() takes once per device with hipGetSymbolAddress.
constexpr int64_t kNoallocCells = (int64_t)1 << 20;  // grid cells: starts take at most 8 MiB
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_base[kMaxDevices] = {};

// Device address of the current device's scratch (looked up on the first call per device).
gq_status scratch_base(unsigned char** out) {
  int dev = -1;
  NA_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return gq::set_error(GQ_EDEVICE, "device index beyond 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_base[dev]) {
    void* p = nullptr;
    NA_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return gq::set_error(GQ_EDEVICE, "hipGetSymbolAddress gave no scratch address");
    g_scratch_base[dev] = (unsigned char*)p;
  }
  *out = g_scratch_base[dev];
  return GQ_OK;
}

}  // namespace

extern "C" gq_status gq_points_near_noalloc(int64_t n_q, const double* q_xyz,
                                            const double* radius, int strict, int64_t n_p,
                                            const double* p_xyz, uint8_t* hit,
                                            void* hip_stream) {
  (void)gq::set_error(GQ_OK, "");
  gq::NearQuery Q;
  bool done = false;
  gq_status st = gq::near_prepare(n_q, q_xyz, radius, n_p, p_xyz, hit, kNoallocCells, Q, done);
  if (st != GQ_OK || done) return st;
  // layout: cell starts, sorted points (x, y, z), queries (x, y, z), radii, hit flags; each
  // segment 256-byte aligned
  const size_t seg[9] = {Q.start.size() * sizeof(int64_t), (size_t)n_p * 8, (size_t)n_p * 8,
                         (size_t)n_p * 8, (size_t)n_q * 8, (size_t)n_q * 8, (size_t)n_q * 8,
                         (size_t)n_q * 8, (size_t)n_q};
  size_t off[9], total = 0;
  for (int i = 0; i < 9; ++i) {
    off[i] = total;
    total += (seg[i] + 255) / 256 * 256;
  }
  if (total > kScratchBytes)
    return gq::set_error(GQ_EINVAL, "gq_points_near_noalloc: the query needs " +
                                        std::to_string(total) + " bytes of device scratch, " +
                                        "more than its fixed " + std::to_string(kScratchBytes));
  unsigned char* base = nullptr;
  st = scratch_base(&base);
  if (st != GQ_OK) return st;
  hipStream_t s = (hipStream_t)hip_stream;
  const void* host[8] = {Q.start.data(), Q.px.data(), Q.py.data(), Q.pz.data(),
                         Q.qx.data(),    Q.qy.data(), Q.qz.data(), radius};
  for (int i = 0; i < 8; ++i)
    NA_HIP(hipMemcpyAsync(base + off[i], host[i], seg[i], hipMemcpyHostToDevice, s));
  auto dp = [&](int i) { return (const double*)(base + off[i]); };
  const gq::AssocCells pts{(const int64_t*)(base + off[0]), dp(1), dp(2), dp(3), nullptr,
                           nullptr, nullptr};
  uint8_t* dhit = base + off[8];
  // the kernel writes every flag, so nothing left by an earlier call needs clearing
  gq::launch_points_near(s, n_q, dp(4), dp(5), dp(6), dp(7), strict, Q.g, pts, dhit);
  NA_HIP(hipGetLastError());
  NA_HIP(hipMemcpyAsync(hit, dhit, n_q, hipMemcpyDeviceToHost, s));
  NA_HIP(hipStreamSynchronize(s));
  return GQ_OK;
}
