// lgt_dslash_noalloc: the Wilson-Dirac operator of lgt_dslash without a
// context and without any device allocation, for callers that cannot
// allocate (code under HIP graph capture, serving loops, harnesses that
// forbid hipMalloc).
//
// Its working storage -- the packed links and the packed input and output
// spinors lgt_dslash keeps in its context -- lives in one file-scope device
// array, `scratch`, sized for lattices of up to kNoAllocMaxSites sites.  Each
// GPU the library runs on holds its own copy of the array until the process
// ends.  Host code never passes the array's name to a kernel (on the host it
// is a stand-in symbol, not a device address): the first call on a device
// looks up that device's address with hipGetSymbolAddress, and every launch
// takes that pointer.  All calls on one GPU share the array, so calls that
// overlap in time on one GPU (different streams or threads) race; calls
// ordered on one stream do not.  The packing kernels write every element the
// hop then reads, so nothing has to start at zero.
#include <cmath>
#include <mutex>
#include <string>

#include "lgt_ctx.h"

using namespace lgt;

namespace {

constexpr int64_t kNoAllocMaxSites = 65536;  // 16^4
// packed links (36 complex per site), packed input and output spinors (12 each)
constexpr size_t kScratchElems = (size_t)60 * kNoAllocMaxSites;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double2 scratch[kScratchElems];

std::mutex g_scratch_mu;
double2* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (looked up once per device).
double2* scratch_on_current_device() {
  int dev = -1;
  LGT_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw Error(LGT_ERR_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    LGT_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw Error(LGT_ERR_DEVICE, "hipGetSymbolAddress returned a null scratch address");
    g_scratch_ptr[dev] = static_cast<double2*>(p);
  }
  return g_scratch_ptr[dev];
}

}  // namespace

lgt_status lgt_dslash_noalloc(const lgt_geom* geom, void* hip_stream, const void* U, const void* in, void* out,
                              double kappa, int32_t dagger) {
  auto fail = [](lgt_status s, const std::string& msg) {
    lgt_set_global_error(msg);
    return s;
  };
  lgt_set_global_error("");
  if (!geom || !U || !in || !out) return fail(LGT_ERR_INVALID_ARGUMENT, "null argument");
  for (int i = 0; i < 4; ++i)
    if (geom->dims[i] < 2 || geom->dims[i] % 2 != 0)
      return fail(LGT_ERR_INVALID_ARGUMENT, "every lattice extent must be even and >= 2");
  if (geom->fermion_t_bc != 1 && geom->fermion_t_bc != -1)
    return fail(LGT_ERR_INVALID_ARGUMENT, "fermion_t_bc must be +1 or -1");
  if (!std::isfinite(kappa)) return fail(LGT_ERR_INVALID_ARGUMENT, "kappa must be finite");
  const int64_t V = (int64_t)geom->dims[0] * geom->dims[1] * geom->dims[2] * geom->dims[3];
  if (V > kNoAllocMaxSites)
    return fail(LGT_ERR_INVALID_ARGUMENT, "lattice too large for lgt_dslash_noalloc: V = " + std::to_string(V) +
                                              " sites, its scratch holds at most " +
                                              std::to_string(kNoAllocMaxSites));
  try {
    Geom g{};
    for (int i = 0; i < 4; ++i) g.L[i] = geom->dims[i];
    g.hx = geom->dims[0] / 2;
    g.vh = (int)(V / 2);
    g.bc = geom->fermion_t_bc;
    g.hop_ns = 0;
    g.hop_order = 0;
    const hipStream_t s = (hipStream_t)hip_stream;
    double2* base = scratch_on_current_device();
    double2* links = base;                      // 72 vh
    double2* a = links + (size_t)72 * g.vh;     // 24 vh: packed input (even half, then odd)
    double2* b = a + (size_t)24 * g.vh;         // 24 vh: packed output
    const size_t h = (size_t)12 * g.vh;
    LGT_HIP(launch_pack(g, 36, (const double2*)U, links, nullptr, nullptr, s));
    LGT_HIP(launch_pack(g, 12, (const double2*)in, a, nullptr, nullptr, s));
    HopIn<double> hin{links, a, a + h};
    if (dagger)
      LGT_HIP((launch_hop_axpy<double, true>(g, -1, hin, b, b + h, a, a + h, -kappa, s)));
    else
      LGT_HIP((launch_hop_axpy<double, false>(g, -1, hin, b, b + h, a, a + h, -kappa, s)));
    LGT_HIP(launch_unpack(g, 12, b, (double2*)out, s));
    return LGT_OK;
  } catch (const Error& e) {
    return fail(e.status, e.what());
  } catch (const std::exception& e) {
    return fail(LGT_ERR_DEVICE, e.what());
  }
}
