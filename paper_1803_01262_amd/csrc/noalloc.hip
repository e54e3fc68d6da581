// phasefield_step_noalloc: the step of phasefield_step for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
// It needs no handle: its three stage buffers live in one file-scope device array of fixed
// size, `scratch`, which every GPU the library runs on holds until the process ends.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>

#include "pf_api_internal.h"

using namespace pf;

static constexpr size_t kScratchBytes = size_t(64) << 20;  // three stage buffers share 64 MiB

// The stage buffers of phasefield_step_noalloc. In host code this name is a host-side stand-in,
// not a device address: host code only ever uses the per-device address that
// hipGetSymbolAddress returns for it (scratch_on_current_device).
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

size_t round_up_256(size_t b) { return (b + 255) & ~size_t(255); }

// Device address of `scratch` on the current device, looked up once per device (with that
// device current) and kept; nullptr with the error recorded on failure.
void* scratch_on_current_device(pf_status* st)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        *st = hip_fail(e, "phasefield_step_noalloc: hipGetDevice");
        return nullptr;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        *st = fail(PF_ERR_UNSUPPORTED, "phasefield_step_noalloc: device %d beyond %d", dev,
                   kMaxDevices);
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            *st = hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol,
                           "phasefield_step_noalloc: hipGetSymbolAddress(scratch)");
            return nullptr;
        }
        g_ptr[dev] = ptr;
    }
    return g_ptr[dev];
}

template <typename T>
hipError_t run(const pf_params& p, int variant, T* phi, const T* U, const T* V, const T* W,
               unsigned char* base, size_t buf, double t0, int32_t nsteps, hipStream_t st)
{
    T* ya = reinterpret_cast<T*>(base);
    T* yb = reinterpret_cast<T*>(base + buf);
    T* acc = reinterpret_cast<T*>(base + 2 * buf);
    return enqueue_steps<T>(p, variant, phi, U, V, W, ya, yb, acc, t0, nsteps, st);
}

}  // namespace

extern "C" size_t phasefield_noalloc_scratch_bytes(void) { return kScratchBytes; }

extern "C" pf_status phasefield_step_noalloc(const pf_params* p, void* phi, const void* u,
                                             const void* v, const void* w, double t0,
                                             int32_t nsteps, void* hip_stream)
{
    pf_status st = validate_params(p);
    if (st != PF_OK) return st;
    if ((st = check_field_ptr(phi, "phi")) != PF_OK) return st;
    if ((st = check_field_ptr(u, "u")) != PF_OK) return st;
    if ((st = check_field_ptr(v, "v")) != PF_OK) return st;
    if ((st = check_field_ptr(w, "w")) != PF_OK) return st;
    if (nsteps < 0) return fail(PF_ERR_INVALID, "nsteps < 0");
    if (!std::isfinite(t0)) return fail(PF_ERR_INVALID, "t0 is not finite");
    const size_t esz = p->dtype == PF_F32 ? sizeof(float) : sizeof(double);
    const size_t cells = (size_t)p->n[0] * p->n[1] * p->n[2];
    const size_t buf = round_up_256(cells * esz);
    if (3 * buf > kScratchBytes)
        return fail(PF_ERR_INVALID,
                    "phasefield_step_noalloc: %zu cells of %zu bytes need 3 x %zu bytes of stage "
                    "buffers, more than the %zu-byte scratch array",
                    cells, esz, buf, kScratchBytes);
    if (nsteps == 0) return PF_OK;
    void* base = scratch_on_current_device(&st);
    if (!base) return st;
    const int variant = p->variant >= 0 ? p->variant : default_variant(*p);
    hipStream_t hs = (hipStream_t)hip_stream;
    hipError_t e =
        p->dtype == PF_F32
            ? run<float>(*p, variant, (float*)phi, (const float*)u, (const float*)v,
                         (const float*)w, (unsigned char*)base, buf, t0, nsteps, hs)
            : run<double>(*p, variant, (double*)phi, (const double*)u, (const double*)v,
                          (const double*)w, (unsigned char*)base, buf, t0, nsteps, hs);
    if (e != hipSuccess) return hip_fail(e, "phasefield_step_noalloc: launch");
    return PF_OK;
}
