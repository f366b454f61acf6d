// Host-only argument checks of the C ABI. No HIP calls: every rule here can
// be exercised without a GPU (the library runs them before enqueueing work).
#pragma once

#include <math.h>
#include <stdint.h>

#include <string>

#include "../../include/tdse.h"

namespace tdse {

constexpr int32_t TAYLOR_MAX_ORDER = 32;
constexpr int32_t LANCZOS_MAX_DIM = 64;
constexpr int64_t MAX_STATES = (int64_t)1 << 40;

inline tdse_status validate_create(const void *out, const void *energies, const void *dipole,
                                   int32_t lmax, int32_t n, int32_t batch, std::string *why) {
    if (!out) { *why = "out is NULL"; return TDSE_E_INVAL; }
    if (!energies) { *why = "energies is NULL"; return TDSE_E_INVAL; }
    if (lmax < 0) { *why = "lmax must be >= 0"; return TDSE_E_INVAL; }
    if (n < 1) { *why = "n must be >= 1"; return TDSE_E_INVAL; }
    if (batch < 1) { *why = "batch must be >= 1"; return TDSE_E_INVAL; }
    if (lmax > 0 && !dipole) { *why = "dipole is NULL with lmax > 0"; return TDSE_E_INVAL; }
    if ((int64_t)(lmax + 1) * n > MAX_STATES / batch) {
        *why = "problem too large ((lmax+1)*n*batch exceeds 2^40)";
        return TDSE_E_INVAL;
    }
    return TDSE_OK;
}

inline tdse_status validate_propagate(bool have_plan, int method, int32_t order, double dt,
                                      int64_t nsteps, bool have_ckpt, int32_t ckpt_every,
                                      std::string *why) {
    if (!have_plan) { *why = "plan is NULL"; return TDSE_E_INVAL; }
    if (method != TDSE_RK4 && method != TDSE_TAYLOR && method != TDSE_LANCZOS && method != TDSE_RKF45) {
        *why = "unknown method";
        return TDSE_E_INVAL;
    }
    if (method == TDSE_TAYLOR && (order < 1 || order > TAYLOR_MAX_ORDER)) {
        *why = "taylor_order must be in [1, 32]";
        return TDSE_E_INVAL;
    }
    if (method == TDSE_LANCZOS && (order < 1 || order > LANCZOS_MAX_DIM)) {
        *why = "the Krylov dimension (taylor_order) must be in [1, 64]";
        return TDSE_E_INVAL;
    }
    if (!(dt > 0.0) || !isfinite(dt)) { *why = "dt must be finite and > 0"; return TDSE_E_INVAL; }
    if (nsteps < 0) { *why = "nsteps must be >= 0"; return TDSE_E_INVAL; }
    if (have_ckpt && ckpt_every < 1) { *why = "ckpt_every must be >= 1 when ckpt is given"; return TDSE_E_INVAL; }
    return TDSE_OK;
}

}  // namespace tdse
