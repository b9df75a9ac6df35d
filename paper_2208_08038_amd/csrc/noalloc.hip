// noalloc.hip -- pic_rho_static: the charge density of pic_rho computed in
// a file-scope device array instead of context scratch, for callers that
// cannot allocate device memory at the time of the call.
//
// The array (`scratch`, kStaticRhoValues FP64 values, 32 MiB) lives in the
// library's code object: every GPU the library runs on holds its own copy
// until the process ends.  Host code never uses the array's name as an
// address: its device address is looked up once per device with
// hipGetSymbolAddress (with that device current) and kept in g_scratch.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "ctx.h"

namespace {

constexpr size_t kStaticRhoValues = size_t(1) << 22;
constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) double scratch[kStaticRhoValues];

namespace {

std::mutex g_mu;
double* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on its
// first use there).
int static_scratch(pic_ctx* c, int dev, double** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(c, PIC_EINVAL, "device id out of range");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(c, PIC_EHIP,
                  std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch[dev] = static_cast<double*>(p);
  }
  *out = g_scratch[dev];
  return PIC_OK;
}

template <typename Real>
int rho_static_t(pic_ctx* c, double* rho, double* plane) {
  const GridInfo& g = c->g;
  // a kernel clears the plane (no memset node, should a caller capture this)
  pic::launch_zero<double>(plane, g.plane, c->stream);
  for (auto& s : c->sp) launch_rho_species<Real>(c, *s, plane);
  pic::launch_fold_periodic_f64(g, plane, c->stream);
  // interior rows straight to the caller's array, one 2D copy per z layer
  const size_t nx = (size_t)g.n[0];
  for (int k = 0; k < g.n[2]; k++) {
    const double* src = plane + g.origin + (int64_t)k * g.sz;
    HIPCHK(c, hipMemcpy2DAsync(rho + (size_t)k * nx * g.n[1], nx * sizeof(double), src,
                               (size_t)g.sy * sizeof(double), nx * sizeof(double),
                               (size_t)g.n[1], hipMemcpyDeviceToHost, c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return PIC_OK;
}

}  // namespace

extern "C" {

int pic_rho_static(pic_ctx* c, double* rho) {
  if (!c || !rho) return c ? fail(c, PIC_EINVAL, "null argument") : PIC_EINVAL;
  if ((size_t)c->g.plane > kStaticRhoValues)
    return fail(c, PIC_EINVAL,
                "grid too large for pic_rho_static: the guarded grid holds " +
                    std::to_string(c->g.plane) + " nodes, at most " +
                    std::to_string(kStaticRhoValues));
  int dev = -1;
  HIPCHK(c, hipGetDevice(&dev));
  if (dev != c->device)
    return fail(c, PIC_ESTATE, "pic_rho_static needs the context's device to be current");
  double* plane = nullptr;
  int rc = static_scratch(c, dev, &plane);
  if (rc) return rc;
  return c->prec == 32 ? rho_static_t<float>(c, rho, plane) : rho_static_t<double>(c, rho, plane);
}

}  // extern "C"
