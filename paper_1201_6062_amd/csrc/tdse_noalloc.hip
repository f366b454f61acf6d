// tdse_propagate_noalloc: the single-vector RK4 / Taylor propagation of
// tdse_propagate with its per-call scratch -- the state vectors and product
// partials of both launch parities and the call descriptor -- in one fixed
// device array of this library instead of the plan's own allocation, and
// without captured graphs. It performs no device allocation and instantiates
// no graph, for callers that cannot allocate (code under HIP graph capture,
// tight serving loops).
//
// The array is a file-scope __device__ symbol. In host code its name is only
// a host-side stand-in, so its device address is taken once per device with
// hipGetSymbolAddress (with that device current, on the first call there) and
// only that address is handed to kernels. Every call on one device shares the
// array: calls that overlap on one device (other streams, other threads) race
// on it, and the array keeps the last call's contents -- the start kernel of
// each call re-initialises everything the launches read first (states of the
// starting parity and its partials).
#include <mutex>

#include "tdse_internal.h"
#include "tdse_validate.h"

namespace tdse {

constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)16 << 20;  // 16 MiB per device
constexpr int NOALLOC_MAX_DEVICES = 64;

static __device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static char *g_scratch_ptr[NOALLOC_MAX_DEVICES];

// Device address of this device's copy of the array (looked up once per device).
static tdse_status scratch_for_device(int dev, char **out) {
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(TDSE_E_UNSUPPORTED, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress of the scratch array");
        }
        g_scratch_ptr[dev] = static_cast<char *>(p);
    }
    *out = g_scratch_ptr[dev];
    return TDSE_OK;
}

}  // namespace tdse

using namespace tdse;

extern "C" tdse_status tdse_propagate_noalloc(tdse_plan p, tdse_method method, int32_t order, double dt,
                                              int64_t nsteps, const double *field, const double *c0, double *cT,
                                              double *ckpt, int32_t ckpt_every, void *stream) {
    clear_error();
    std::string why;
    tdse_status st = validate_propagate(p != nullptr, (int)method, order, dt, nsteps, ckpt != nullptr, ckpt_every,
                                        &why);
    if (st != TDSE_OK) return fail(st, why);
    if (method != TDSE_RK4 && method != TDSE_TAYLOR)
        return fail(TDSE_E_UNSUPPORTED, "tdse_propagate_noalloc covers RK4 and Taylor-p");
    if (p->batch != 1) return fail(TDSE_E_UNSUPPORTED, "tdse_propagate_noalloc needs a batch-1 plan");
    int dev = -1;
    TDSE_HIP(hipGetDevice(&dev));
    if (dev != p->device) return fail(TDSE_E_INVAL, "the plan's device must be the current device");
    if (nsteps > 0 && (st = check_device_ptr(field, "field"))) return st;
    if ((st = check_device_ptr(c0, "c0")) || (st = check_device_ptr(cT, "cT"))) return st;
    if (ckpt && (st = check_device_ptr(ckpt, "ckpt"))) return st;
    const int m = method == TDSE_RK4 ? 4 : order;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (p->small)  // one workgroup, state in LDS: no scratch at all
        return vec_propagate_on(p, p->vb, false, method, m, dt, nsteps, field, c0, cT, ckpt, ckpt_every, s);
    const size_t need = vec_scratch_bytes(p->lmax, p->n, p->T);
    if (need > NOALLOC_SCRATCH_BYTES)
        return fail(TDSE_E_UNSUPPORTED, "problem needs " + std::to_string(need) + " bytes of scratch, more than the " +
                                             std::to_string(NOALLOC_SCRATCH_BYTES) + " of the fixed array");
    char *base = nullptr;
    if ((st = scratch_for_device(dev, &base))) return st;
    VecBuffers vb = p->vb;  // the plan's Hamiltonian, the fixed array's per-call buffers
    vec_bind_scratch(vb, base, p->lmax, p->n, p->T);
    return vec_propagate_on(p, vb, false, method, m, dt, nsteps, field, c0, cT, ckpt, ckpt_every, s);
}
