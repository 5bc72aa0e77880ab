// psim_amplitudes_static: amplitudes with the workspace in a fixed device
// array of the library, for callers that cannot allocate device memory.
//
// The array below is the workspace of the row sweep (trie tables, boundaries,
// intermediates) or of the square partition, exactly as the caller's
// workspace is for psim_amplitudes; the same kernels run on it.  Host code
// never passes the array's name to a kernel or a copy: its device address is
// looked up once per device (hipGetSymbolAddress, with that device current)
// and that address is used everywhere.  Every call on one device shares the
// array and leaves its contents behind; everything the sweep reads is written
// earlier in the same call (tables uploaded, boundaries produced with beta =
// 0, row maxima cleared by a fill kernel), so nothing needs clearing between
// calls.  Calls that overlap on one device race on the array.
#include <hip/hip_runtime.h>

#include <mutex>
#include <new>
#include <string>

#include "psim_internal.hpp"

using namespace psim;

namespace {

__device__ __align__(256) char scratch[PSIM_STATIC_WORKSPACE_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};  // device address of `scratch` per device ordinal

// Device address of the array on `device` (made current by the caller).
void* scratch_address(int device) {
  if (device < 0 || device >= kMaxDevices) fail(PSIM_EINVAL, "device ordinal out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[device]) {
    void* p = nullptr;
    hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(static workspace)");
    if (!p) fail(PSIM_EDEVICE, "hipGetSymbolAddress returned NULL for the static workspace");
    g_scratch[device] = p;
  }
  return g_scratch[device];
}

}  // namespace

extern "C" psim_status psim_amplitudes_static(psim_plan_t* pl, const uint8_t* bits, size_t n, void* hip_stream,
                                              double* out_amp, double* out_rel_err) {
  try {
    if (!pl) fail(PSIM_EINVAL, "plan is NULL");
    if (pl->host_only) fail(PSIM_EINVAL, "plan was made with PSIM_PLAN_HOST_ONLY");
    if (pl->ws_total > (uint64_t)PSIM_STATIC_WORKSPACE_BYTES)
      fail(PSIM_EINVAL, "plan needs " + std::to_string(pl->ws_total) + " bytes of workspace; the static "
                        "workspace holds " + std::to_string((uint64_t)PSIM_STATIC_WORKSPACE_BYTES) +
                        " (use psim_amplitudes with a caller-owned workspace, or a smaller max_batch)");
    hip_check(hipSetDevice(pl->opts.device), "hipSetDevice");
    void* ws = scratch_address(pl->opts.device);
    run_amplitudes(pl, bits, n, ws, (size_t)PSIM_STATIC_WORKSPACE_BYTES, hip_stream, out_amp, true, out_rel_err);
    return PSIM_OK;
  } catch (const Error& e) {
    set_last_error(e.msg);
    return e.status;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return PSIM_ENOMEM;
  } catch (const std::exception& e) {
    set_last_error(std::string("internal error: ") + e.what());
    return PSIM_EINTERNAL;
  } catch (...) {
    set_last_error("internal error");
    return PSIM_EINTERNAL;
  }
}
