// C ABI of the TDSE library: argument checking, plan lifetime, scheduling of
// the per-product launches, and graph capture of step chunks.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "tdse_internal.h"
#include "tdse_stability.h"
#include "tdse_validate.h"

namespace tdse {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }
tdse_status fail(tdse_status st, const std::string &msg) {
    g_last_error = msg;
    return st;
}
tdse_status hip_fail(hipError_t e, const char *what) {
    g_last_error = std::string("HIP error ") + hipGetErrorString(e) + " in " + what;
    return TDSE_E_HIP;
}

// Device memory check used by every entry point before anything is enqueued.
static bool is_device_ptr(const void *p) {
    if (!p) return false;
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

static tdse_status check_dev(const void *p, const char *name) {
    if (!p) return fail(TDSE_E_INVAL, std::string(name) + " is NULL");
    if (reinterpret_cast<uintptr_t>(p) % 8) return fail(TDSE_E_INVAL, std::string(name) + " is not 8-byte aligned");
    if (!is_device_ptr(p)) return fail(TDSE_E_INVAL, std::string(name) + " is not device memory");
    return TDSE_OK;
}

tdse_status check_device_ptr(const void *p, const char *name) { return check_dev(p, name); }

// max |E| and the largest absolute row sum of the coupling (an upper bound of
// its spectral norm), from device copies of the energies and of the row-major
// blocks (dip may be NULL when lmax == 0). Synchronises s.
static tdse_status coupling_bounds(tdse_plan p, const double *en, const double *dip, hipStream_t s) {
    const size_t ns = (size_t)(p->lmax + 1) * p->n;
    std::vector<double> hen(ns), hrs(ns, 0.0);
    double *rs = nullptr;
    hipError_t e = hipSuccess;
    if (p->lmax > 0) {
        e = hipMalloc(&rs, ns * sizeof(double));
        if (e == hipSuccess) e = coupling_rowsum(dip, p->lmax, p->n, rs, s);
        if (e == hipSuccess) e = hipMemcpyAsync(hrs.data(), rs, ns * sizeof(double), hipMemcpyDeviceToHost, s);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(hen.data(), en, ns * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (rs) (void)hipFree(rs);
    if (e != hipSuccess) return hip_fail(e, "spectrum bounds of the plan");
    double emax = 0.0, dmax = 0.0;
    for (size_t g = 0; g < ns; ++g) {
        emax = fabs(hen[g]) > emax ? fabs(hen[g]) : emax;
        dmax = hrs[g] > dmax ? hrs[g] : dmax;
    }
    p->emax = emax;
    p->dnorm = dmax;
    return TDSE_OK;
}

// ---------------------------------------------------------------------------
// Launch schedule of one step: the completion each launch performs on the
// previous launch's product (see vec_kernels.hip).
static void step_launches(tdse_method m, int order, std::vector<Completion> &out) {
    out.clear();
    if (m == TDSE_RK4) {
        // launch 1 completes stage 4 of the previous step, launches 2..4 complete stages 1..3
        out.push_back({CK_RK4_END, 2, -1, 0, 1.0 / 6.0, 0.0});
        out.push_back({CK_RK4_MID, 0, 0, 1, 1.0 / 6.0, 0.5});
        out.push_back({CK_RK4_MID, 1, 0, 0, 2.0 / 6.0, 0.5});
        out.push_back({CK_RK4_MID, 1, 0, 0, 2.0 / 6.0, 1.0});
    } else {
        // launch 1 completes term p of the previous step, launch m completes term m-1
        out.push_back({CK_TAY_END, 0, -1, 0, 0.0, 1.0 / order});
        for (int t = 1; t < order; ++t) out.push_back({CK_TAY_MID, 0, 0, 0, 0.0, 1.0 / t});
    }
}

static Completion final_completion(tdse_method m, int order) {
    std::vector<Completion> v;
    step_launches(m, order, v);
    return v[0];
}

static hipError_t enqueue_steps(tdse_plan p, const VecBuffers &vb, tdse_method m, int order, int64_t nsteps_chunk,
                                int32_t &parity, hipStream_t s) {
    std::vector<Completion> sl;
    step_launches(m, order, sl);
    for (int64_t k = 0; k < nsteps_chunk; ++k) {
        for (const Completion &c : sl) {
            VecLaunch L{};
            L.comp = c;
            L.off = (int32_t)k;
            L.parity = parity;
            L.slots = m == TDSE_RK4 ? 3 : 1;
            hipError_t e;
            if (p->lmax == 0) {
                e = vec_launch_combine(vb, L, s);
            } else if (p->split) {
                L.np = patch_np(p->T);  // partials of the preceding patch products launch (zeros at the start)
                e = vec_launch_combine(vb, L, s);
                if (e == hipSuccess) e = vec_launch_products(vb, L, s);
            } else {
                e = vec_launch_tiles(vb, L, s);
            }
            if (e != hipSuccess) return e;
            parity ^= 1;
        }
    }
    return hipSuccess;
}


static tdse_status get_chunk_graph(tdse_plan p, tdse_method m, int order, hipGraphExec_t *out) {
    char key[64];
    snprintf(key, sizeof key, "vec:%d:%d:%d", (int)m, order, CHUNK_STEPS);
    auto it = p->graphs.find(key);
    if (it != p->graphs.end()) {
        *out = it->second;
        return TDSE_OK;
    }
    hipStream_t cs;
    TDSE_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    int32_t par = 0;
    if (e == hipSuccess) e = enqueue_steps(p, p->vb, m, order, CHUNK_STEPS, par, cs);
    hipError_t e2 = hipStreamEndCapture(cs, &g);
    if (e == hipSuccess) e = e2;
    hipGraphExec_t ge = nullptr;
    if (e == hipSuccess) e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(e, "graph capture of a step chunk");
    }
    p->graphs[key] = ge;
    p->graph_defs.push_back(g);
    *out = ge;
    return TDSE_OK;
}

static bool graphs_enabled() {
    const char *v = getenv("TDSE_NO_GRAPH");
    return !(v && v[0] == '1');
}

}  // namespace tdse

// Single-vector propagation on the buffers vb (the plan's own, or the fixed
// scratch array of tdse_propagate_noalloc); use_graphs: whole 64-step chunks
// replay the plan's captured graph (only for the plan's own buffers, which
// the graph was captured with).
tdse_status tdse::vec_propagate_on(tdse_plan p, const VecBuffers &vb, bool use_graphs, tdse_method m, int order,
                                   double dt, int64_t nsteps, const double *field, const double *c0, double *cT,
                                   double *ckpt, int32_t K, hipStream_t s) {
    if (p->small) {
        TDSE_HIP(small_propagate(p->en, p->dip, p->gauge, p->lmax, p->n, (int)m, order, dt, nsteps, field, c0, cT, ckpt,
                                 ckpt ? K : 1, s));
        return TDSE_OK;
    }
    CallDesc d{};
    d.base_step = 0;
    d.nsteps = nsteps;
    d.field = field;
    d.ckpt = ckpt;
    d.ckpt_every = ckpt ? K : 1;
    d.dt = dt;
    d.slots = m == TDSE_RK4 ? 3 : 1;
    TDSE_HIP(set_desc(vb.desc, d, s));
    int32_t parity = 0;
    TDSE_HIP(vec_launch_start(vb, parity, c0, m, s));
    hipGraphExec_t ge = nullptr;
    if (use_graphs && graphs_enabled() && nsteps >= CHUNK_STEPS) {
        tdse_status st = get_chunk_graph(p, m, order, &ge);
        if (st != TDSE_OK) return st;
    }
    int64_t base = 0;
    TDSE_HIP(chunk_begin(vb.desc, 0, s));
    for (int64_t done = 0; done < nsteps; done += CHUNK_STEPS) {
        base = done;
        if (done > 0) TDSE_HIP(chunk_begin(vb.desc, done, s));
        const int64_t len = nsteps - done < CHUNK_STEPS ? nsteps - done : CHUNK_STEPS;
        if (ge && len == CHUNK_STEPS) {
            TDSE_HIP(hipGraphLaunch(ge, s));  // even launch count: parity unchanged
        } else {
            TDSE_HIP(enqueue_steps(p, vb, m, order, len, parity, s));
        }
    }
    VecLaunch L{};
    L.comp = final_completion(m, order);
    L.off = (int32_t)(nsteps - base);
    L.parity = parity;
    L.slots = m == TDSE_RK4 ? 3 : 1;
    L.finish = 1;
    L.np = p->split && p->lmax > 0 ? patch_np(p->T) : 0;
    L.out = cT;
    TDSE_HIP(vec_launch_combine(vb, L, s));
    return TDSE_OK;
}

namespace tdse {

static tdse_status vec_propagate(tdse_plan p, tdse_method m, int order, double dt, int64_t nsteps,
                                 const double *field, const double *c0, double *cT, double *ckpt,
                                 int32_t K, hipStream_t s) {
    return vec_propagate_on(p, p->vb, true, m, order, dt, nsteps, field, c0, cT, ckpt, K, s);
}

size_t vec_scratch_bytes(int lmax, int n, int T) {
    const size_t ns = (size_t)(lmax + 1) * n;
    const size_t npart = (size_t)lmax * T * T * VEC_TILE_MAX;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    return 6 * al(ns * sizeof(double2)) + 4 * al(npart * sizeof(double2)) + al(sizeof(CallDesc));
}

// Point the per-call buffers of vb (states of both parities, partials of both
// parities, the call descriptor) into one region of vec_scratch_bytes bytes.
void vec_bind_scratch(VecBuffers &vb, char *base, int lmax, int n, int T) {
    const size_t ns = (size_t)(lmax + 1) * n;
    const size_t npart = (size_t)lmax * T * T * VEC_TILE_MAX;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t st_bytes = al(ns * sizeof(double2)), part_bytes = al(npart * sizeof(double2));
    size_t off = 0;
    for (int par = 0; par < 2; ++par)
        for (int v = 0; v < 3; ++v) {
            vb.side[par].st[v] = reinterpret_cast<double2 *>(base + off);
            off += st_bytes;
        }
    for (int par = 0; par < 2; ++par) {
        vb.side[par].rowp = reinterpret_cast<double2 *>(base + off);
        off += part_bytes;
        vb.side[par].colp = reinterpret_cast<double2 *>(base + off);
        off += part_bytes;
    }
    vb.desc = reinterpret_cast<CallDesc *>(base + off);
}

// Lay the plan's scratch out in one allocation.
static tdse_status vec_alloc(tdse_plan p) {
    const size_t total = vec_scratch_bytes(p->lmax, p->n, p->T);
    char *base = nullptr;
    if (hipMalloc(&base, total) != hipSuccess) {
        (void)hipGetLastError();
        return fail(TDSE_E_NOMEM, "hipMalloc of plan scratch failed");
    }
    p->scratch = reinterpret_cast<double *>(base);
    p->scratch_bytes = total;
    vec_bind_scratch(p->vb, base, p->lmax, p->n, p->T);
    p->vb.en = p->en;
    p->vb.dip = p->dip;
    p->vb.lmax = p->lmax;
    p->vb.n = p->n;
    p->vb.ld = p->ld;
    p->vb.T = p->T;
    p->vb.gauge = p->gauge;
    return TDSE_OK;
}

// ---------------------------------------------------------------------------
// Batched path.

// Tile shape for a batched plan.
//  * 2B <= 64 real columns (up to 32 pulses): the small-batch kernel (K
//    split over eight waves, operands straight into registers; ks = 8),
//    32-row tiles over all columns.
//  * otherwise TN from the padded column count and TM the largest of
//    128/64/32 that still gives >= 512 workgroups (two per CU); grids short
//    of that take K chunks of 32 and two K groups per workgroup.
// A tuned (cache) or forced ($TDSE_TILE="TMxTNxKC[xKS]") choice overrides;
// $TDSE_KGROUPS=1/2 overrides the K groups of the LDS kernels, and
// $TDSE_SKINNY=0 turns the small-batch kernel off.
static void bat_pick_tile(int lmax, int n, int batch, const TileChoice *force, int *tm, int *tn, int *kc,
                          int *ks) {
    const int ldu = ((2 * batch + 31) / 32) * 32;
    *tn = ldu % 64 == 0 ? 64 : 32;
    *tm = 32;
    *kc = 32;  // grids short of two workgroups per CU even at TM = 32: longer K
               // chunks, fewer barriers (32 pulses at Lmax=15, N=500: 40 vs 48 us per stage)
    for (int cand : {128, 64, 32}) {
        const int np = ((n + cand - 1) / cand) * cand;
        if ((long)(lmax + 1) * (np / cand) * (ldu / *tn) >= 512) {
            *tm = cand;
            *kc = 16;
            break;
        }
    }
    if (*tn != 64) *kc = 16;  // compiled K-chunk-32 shapes have TN = 64 or 128
    // such grids also get two K groups (eight waves) per workgroup
    *ks = *kc == 32 || (*tm == 32 && *tn == 32) ? 2 : 1;
    const char *sk = getenv("TDSE_SKINNY");
    if (2 * batch <= 64 && !(sk && sk[0] == '0')) {
        *tm = 32;
        *tn = 2 * batch <= 32 ? 32 : 64;
        *kc = 16;
        *ks = 8;
    }
    TileChoice tc{0, 0, 0, 0, 0};
    if (force) tc = *force;
    else tune_lookup(lmax, n, batch, &tc);
    if (tc.tm > 0 || tc.tn > 0 || tc.kc > 0) *ks = tc.ks > 0 ? tc.ks : 1;  // a forced or tuned shape
    if (tc.tm > 0) *tm = tc.tm;
    if (tc.tn > 0) *tn = tc.tn;
    if (tc.kc > 0) *kc = tc.kc;
    if (const char *kg = getenv("TDSE_KGROUPS")) {
        if (*ks != 8 && kg[0] == '1') *ks = 1;
        if (*ks != 8 && kg[0] == '2') *ks = 2;
    }
    // two K groups exist for 32x64x32 and 32x32x16; the small-batch kernel for 32-row tiles of 32 or 64 columns
    if (*ks == 8 && !(*tm == 32 && (*tn == 32 || *tn == 64) && 2 * batch <= *tn)) *ks = 1;
    if (*ks == 2 && !((*tm == 32 && *tn == 64 && *kc == 32) || (*tm == 32 && *tn == 32 && *kc == 16))) *ks = 1;
}

static tdse_status bat_create(tdse_plan p, const double *energies, const double *dipole,
                              hipStream_t s, const TileChoice *force) {
    BatBuffers &b = p->bb;
    b.gauge = p->gauge;
    b.lmax = p->lmax;
    b.n = p->n;
    b.batch = p->batch;
    bat_pick_tile(p->lmax, p->n, p->batch, force, &b.tm, &b.tn, &b.kc, &b.ks);
    b.np = ((p->n + b.tm - 1) / b.tm) * b.tm;
    b.ldu = ((2 * p->batch + b.tn - 1) / b.tn) * b.tn;
    const size_t ns_pad = (size_t)(p->lmax + 1) * b.np;
    const size_t dsz = (size_t)p->lmax * b.np * b.np;
    const size_t usz = ns_pad * b.ldu;
    const size_t total = ns_pad + 2 * dsz + 4 * usz;
    double *mem = nullptr;
    if (hipMalloc(&mem, total * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(TDSE_E_NOMEM, "hipMalloc of the batched plan failed");
    }
    p->bat_mem = mem;
    b.en = mem;
    b.d = b.en + ns_pad;
    b.dT = b.d + dsz;
    b.u[0] = b.dT + dsz;
    b.u[1] = b.u[0] + usz;
    b.c = b.u[1] + usz;
    b.acc = b.c + usz;
    const size_t ns = (size_t)(p->lmax + 1) * p->n;
    double *stage_en = nullptr, *stage_d = nullptr;
    hipError_t e = hipMalloc(&stage_en, ns * sizeof(double));
    if (e == hipSuccess && p->lmax > 0) e = hipMalloc(&stage_d, (size_t)p->lmax * p->n * p->n * sizeof(double));
    if (e == hipSuccess) e = hipMemcpyAsync(stage_en, energies, ns * sizeof(double), hipMemcpyDefault, s);
    if (e == hipSuccess && p->lmax > 0)
        e = hipMemcpyAsync(stage_d, dipole, (size_t)p->lmax * p->n * p->n * sizeof(double), hipMemcpyDefault, s);
    if (e == hipSuccess) e = hipMemsetAsync(b.u[0], 0, 4 * usz * sizeof(double), s);
    if (e == hipSuccess) e = bat_layout(stage_d, stage_en, b, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    tdse_status st = e == hipSuccess ? coupling_bounds(p, stage_en, stage_d, s) : TDSE_OK;
    if (stage_en) (void)hipFree(stage_en);
    if (stage_d) (void)hipFree(stage_d);
    if (e != hipSuccess) return hip_fail(e, "batched plan setup");
    return st;
}

static void bat_schedule(tdse_method m, int order, std::vector<BatLaunch> &out) {
    out.clear();
    if (m == TDSE_RK4) {
        //            kind        slot first parity w_acc      a_next
        out.push_back({CK_RK4_MID, 0, 1, 0, 1.0 / 6.0, 0.5, 0, 0, 0, 0, 0, 0, 0, nullptr, nullptr});
        out.push_back({CK_RK4_MID, 1, 0, 0, 2.0 / 6.0, 0.5, 0, 0, 0, 0, 0, 0, 0, nullptr, nullptr});
        out.push_back({CK_RK4_MID, 1, 0, 0, 2.0 / 6.0, 1.0, 0, 0, 0, 0, 0, 0, 0, nullptr, nullptr});
        out.push_back({CK_RK4_END, 2, 0, 0, 1.0 / 6.0, 0.0, 0, 0, 0, 0, 0, 0, 0, nullptr, nullptr});
    } else if (m == TDSE_RKF45) {
        for (int st = 0; st < 6; ++st)
            out.push_back({CK_RKF, st, 0, 0, 0.0, 0.0, 0, 0, 0, 0, 0, 0, 0, nullptr, nullptr});
    } else {
        for (int t = 1; t <= order; ++t)
            out.push_back({t == order ? CK_TAY_END : CK_TAY_MID, 0, t == 1 ? 1 : 0, 0, 0.0, 1.0 / t, 0, 0, 0,
                           0, 0, 0, 0, nullptr, nullptr});
    }
}

static int slots_of(tdse_method m) { return m == TDSE_RK4 ? 3 : (m == TDSE_RKF45 ? 6 : 1); }

static tdse_status bat_propagate(tdse_plan p, tdse_method m, int order, double dt, int64_t nsteps,
                                 const double *field, const double *c0, double *cT, double *ckpt,
                                 int32_t K, hipStream_t s, double *err = nullptr) {
    BatBuffers b = p->bb;
    b.field = field;
    double *gp = nullptr;
    const int rowtiles = (b.lmax + 1) * (b.np / b.tm);
    if (m == TDSE_RKF45) {
        // k_1..k_5 and the per-row-tile error partials, kept by the plan
        if (!p->rkf_mem) {
            const size_t usz = (size_t)(b.lmax + 1) * b.np * b.ldu;
            if (hipMalloc(&p->rkf_mem, (5 * usz + (size_t)rowtiles * b.batch) * sizeof(double)) != hipSuccess) {
                (void)hipGetLastError();
                p->rkf_mem = nullptr;
                return fail(TDSE_E_NOMEM, "hipMalloc of the Runge-Kutta-Fehlberg workspace failed");
            }
        }
        b.kst = p->rkf_mem;
        gp = p->rkf_mem + 5 * (size_t)(b.lmax + 1) * b.np * b.ldu;
    }
    TDSE_HIP(bat_pack(b, c0, m == TDSE_TAYLOR ? 1 : 0, s));
    const int rows = ckpt ? (int)(nsteps / K + 1) : 0;
    if (ckpt) TDSE_HIP(bat_ckpt0(b, c0, ckpt, rows, s));
    std::vector<BatLaunch> sched;
    bat_schedule(m, order, sched);
    int parity = 0;
    for (int64_t k = 0; k < nsteps; ++k) {
        for (BatLaunch L : sched) {
            L.parity = parity;
            L.dt = dt;
            L.step = k;
            L.nsteps = nsteps;
            L.slots = slots_of(m);
            if (ckpt && (k + 1) % K == 0) {
                L.ckpt = ckpt;
                L.ckpt_row = (int32_t)((k + 1) / K);
                L.ckpt_rows = rows;
            }
            if (err && L.kind == CK_RKF && L.slot == 5) L.gpart = gp;
            TDSE_HIP(bat_launch_stage(b, L, s));
            parity ^= 1;
        }
        if (err) TDSE_HIP(bat_reduce_err(gp, rowtiles, b.batch, k, nsteps, err, s));
    }
    // the current c lives in b.c whatever the parity
    TDSE_HIP(bat_unpack(b, cT, s));
    return TDSE_OK;
}

static tdse_status bat_hmul(tdse_plan p, const double *fields, const double *u, double *y, hipStream_t s) {
    BatBuffers b = p->bb;
    b.field = fields;
    TDSE_HIP(bat_pack(b, u, 0, s));
    BatLaunch L{};
    L.kind = CK_HMUL;
    L.parity = 0;
    L.dt = 1.0;
    L.step = 0;
    L.nsteps = 1;
    L.slots = 1;
    L.out = y;
    TDSE_HIP(bat_launch_stage(b, L, s));
    return TDSE_OK;
}

// ---------------------------------------------------------------------------
// Short-iterative Lanczos propagation (any plan): the products H v_j run on
// the plan's own kernels, the recurrence and the small exponential in
// lanczos_kernels.hip.

// y = H(field[., k]) u for the plan's pulses (caller layout). Single-vector
// plans read the sample from the chunk staged at `base` by chunk_begin.
static hipError_t lz_product(tdse_plan p, const double *field, int64_t nsteps, int64_t k, int64_t base,
                             const double *u, double *y, double *dotp, const LzNorm *nz, bool products,
                             hipStream_t s) {
    hipError_t e;
    if (p->batch > 1) {
        BatBuffers b = p->bb;
        b.field = field;
        if ((e = bat_pack(b, u, 0, s)) != hipSuccess) return e;
        BatLaunch L{};
        L.kind = CK_HMUL;
        L.parity = 0;
        L.dt = 1.0;
        L.step = k;
        L.nsteps = nsteps;
        L.slots = 1;
        L.out = y;
        return bat_launch_stage(b, L, s);
    }
    // The Krylov vector itself is the product input: the products launch of
    // the split path reads u from the parity-0 state buffers, which this
    // launch's copy of the buffers points at u; the completion launch then
    // forms y = E o u + F z from the partials and u (with nz: u is the
    // unnormalised x_j, which that launch normalises in place).
    VecBuffers vb = p->vb;
    vb.side[0].st[2] = reinterpret_cast<double2 *>(const_cast<double *>(u));
    if (p->lmax > 0 && products) {  // (else the partials come from vec_launch_lz_products)
        VecLaunch P{};
        P.parity = 1;  // reads u from parity 0, writes the partials of parity 0
        P.slots = 1;
        if ((e = vec_launch_products(vb, P, s)) != hipSuccess) return e;
    }
    VecLaunch H{};
    H.comp = {CK_HMUL, 0, 0, 0, 0.0, 0.0};
    H.parity = 0;
    H.slots = 1;
    H.off = (int32_t)(k - base);
    H.np = p->lmax > 0 && products ? patch_np(p->T) : 0;  // patch products, or one partial per tile
    H.out = y;
    return nz ? vec_launch_hmul_dot(vb, H, dotp, *nz, s) : vec_launch_combine(vb, H, s);
}

// The steps of short-iterative Lanczos from k0 (k0 - base: offset in the
// field chunk) on the state c: per step the Krylov basis, m products with the
// recurrence, the small exponential and the recombination. ckpt rows are
// written when ckpt is given.
struct LzWork {
    double *V, *W, *alpha, *beta, *beta0, *y, *C;
    double *dotp, *normp;  // one pulse: per-segment dots, per-workgroup norms
    double *bdot, *bnorm;  // several pulses: per-(row tile, pulse) alpha parts, per-(pulse, chunk) norm parts
    double *qp[2], *ep[2], *np[2];  // one pulse, one launch per product: parts by parity
    size_t vstride;
    int64_t len, ncplx;
};

static hipError_t lz_enqueue_steps(tdse_plan p, const LzWork &w, int m, double dt, const double *dt_dev,
                                   int64_t nsteps, const double *field, int64_t k0, int64_t count, int64_t base,
                                   double *c, double *ckpt, int32_t K, int64_t rows, hipStream_t s) {
    const int B = p->batch;
    hipError_t e = hipSuccess;
    for (int64_t k = k0; k < k0 + count && e == hipSuccess; ++k) {
        const bool row = ckpt && (k + 1) % K == 0;
        // one launch per Krylov product on plans of the fused tile path (at
        // most 512 tiles; the split path's plans re-read fewer partials with
        // separate product and completion launches)
        if (B == 1 && p->lmax > 0 && !p->split && (int64_t)p->lmax * p->T * p->T <= 512) {
            if (k == k0) e = lz_begin_wide(c, w.V, w.normp, w.ncplx, s);  // x_0 = c
            const double *fs = reinterpret_cast<const double *>(reinterpret_cast<const char *>(p->vb.desc) +
                                                                offsetof(CallDesc, chunk_field)) +
                               (k - base) + 1;
            for (int j = 0; j < m && e == hipSuccess; ++j) {
                const int pw = j & 1, pr = pw ^ 1;
                LzFused f{};
                f.xprev = w.V + (size_t)(j > 0 ? j - 1 : 0) * w.vstride;
                f.xprev2 = w.V + (size_t)(j > 1 ? j - 2 : 0) * w.vstride;
                f.xout = w.V + (size_t)j * w.vstride;
                f.qin = w.qp[pr];
                f.ein = w.ep[pr];
                f.nin = w.np[pr];
                f.qout = w.qp[pw];
                f.eout = w.ep[pw];
                f.nout = w.np[pw];
                f.fsample = fs;
                f.alpha = w.alpha;
                f.beta = w.beta;
                f.beta0 = w.beta0;
                f.k = j;
                e = vec_launch_lz_fused(p->vb, f, s);
            }
            const int pl = (m - 1) & 1;
            if (e == hipSuccess)
                e = lz_expm_fused(w.alpha, w.beta, w.beta0, w.qp[pl], w.ep[pl], w.np[pl], 2 * p->lmax * p->T * p->T,
                                  (p->lmax + 1) * p->T, fs, dt, dt_dev, m, w.y, s);
            if (e == hipSuccess)
                e = lz_combine_wide(w.V, w.y, m, w.ncplx, c, row ? ckpt : nullptr, row ? (k + 1) / K : 0, w.normp,
                                    s);
            continue;
        }
        if (B == 1) {  // the recurrence spread over many workgroups
            // x_0 = c with its norm parts; after the first step the previous
            // step's recombination has left both
            if (k == k0) e = lz_begin_wide(c, w.V, w.normp, w.ncplx, s);
            const int nseg = (p->lmax + 1) * p->T;
            for (int j = 0; j < m && e == hipSuccess; ++j) {
                double *vj = w.V + (size_t)j * w.vstride;
                const bool last = j + 1 == m;
                // with dipole blocks the update of step j - 1 runs inside the
                // product launch of x_j, which leaves per-segment norm parts
                const bool folded = p->lmax > 0 && j > 0;
                const LzNorm nz{w.normp, folded ? nseg : lz_wide_groups(w.ncplx), j, w.beta0, w.alpha, w.beta};
                if (folded) {
                    const LzUpdate u{w.dotp, nseg, j - 1, w.W, vj - w.vstride, j > 1 ? vj - 2 * w.vstride : nullptr,
                                     vj, w.alpha, w.beta, w.normp};
                    e = vec_launch_lz_products(p->vb, u, s);
                    if (e == hipSuccess) e = lz_product(p, field, nsteps, k, base, vj, w.W, w.dotp, &nz, false, s);
                } else {
                    e = lz_product(p, field, nsteps, k, base, vj, w.W, w.dotp, &nz, true, s);
                }
                // without dipole blocks a separate update launch
                if (e == hipSuccess && p->lmax == 0)
                    e = lz_update(w.dotp, nseg, vj, j > 0 ? vj - w.vstride : nullptr, w.W,
                                  last ? nullptr : vj + w.vstride, w.alpha, w.beta, j, last ? 1 : 0, w.normp,
                                  w.ncplx, s);
            }
            if (e == hipSuccess)
                e = lz_expm(w.alpha, w.beta, w.beta0, dt, dt_dev, m, B, w.y, p->lmax > 0 ? w.dotp : nullptr, nseg,
                            s);
            if (e == hipSuccess)
                e = lz_combine_wide(w.V, w.y, m, w.ncplx, c, row ? ckpt : nullptr, row ? (k + 1) / K : 0, w.normp,
                                    s);
            continue;
        }
        // several pulses: batched products on the matrix cores (each leaving
        // per-row-tile parts of alpha), the recurrence over many workgroups
        BatBuffers bb = p->bb;
        bb.field = field;
        const int rowtiles = (bb.lmax + 1) * (bb.np / bb.tm);
        e = lzb_norm_parts(c, B, w.len, w.bnorm, s);
        if (e == hipSuccess) e = lzb_normalize(bb, c, w.bnorm, w.V, -1, m, w.alpha, w.beta, w.beta0, w.len, s);
        for (int j = 0; j < m && e == hipSuccess; ++j) {
            const double *vj = w.V + (size_t)j * w.vstride;
            const bool last = j + 1 == m;
            BatLaunch L{};
            L.kind = CK_HMUL;
            L.parity = 0;  // the product input is u[0], written by lzb_normalize
            L.dt = 1.0;
            L.step = k;
            L.nsteps = nsteps;
            L.slots = 1;
            L.out = w.W;
            L.gpart = w.bdot;
            e = bat_launch_stage(bb, L, s);
            if (e == hipSuccess)
                e = lzb_update(w.bdot, rowtiles, vj, j > 0 ? vj - w.vstride : nullptr, w.W, w.alpha, w.beta,
                               w.bnorm, j, m, last ? 1 : 0, B, w.len, s);
            if (e == hipSuccess && !last)
                e = lzb_normalize(bb, w.W, w.bnorm, w.V + (size_t)(j + 1) * w.vstride, j, m, w.alpha, w.beta,
                                  w.beta0, w.len, s);
        }
        if (e == hipSuccess) e = lz_expm(w.alpha, w.beta, w.beta0, dt, dt_dev, m, B, w.y, nullptr, 0, s);
        if (e == hipSuccess)
            e = lz_combine(w.V, w.vstride, w.y, m, B, w.ncplx, c, row ? ckpt : nullptr, rows, row ? (k + 1) / K : 0, s);
    }
    return e;
}

static tdse_status lz_propagate(tdse_plan p, int m, double dt, int64_t nsteps, const double *field,
                                const double *c0, double *cT, double *ckpt, int32_t K, hipStream_t s) {
    const int B = p->batch;
    const int64_t ncplx = (int64_t)(p->lmax + 1) * p->n, len = 2 * ncplx;
    const size_t vstride = (size_t)B * len;
    // V (m vectors), W, the recurrence coefficients and y, and for captured
    // steps a state vector of the plan's own (a graph cannot follow cT)
    const size_t nseg = (size_t)(p->lmax + 1) * (p->T > 0 ? p->T : 1);
    const size_t ntl = (size_t)p->lmax * (p->T > 0 ? p->T : 1) * (p->T > 0 ? p->T : 1);
    const size_t nbdot = B > 1 ? (size_t)(p->lmax + 1) * (p->bb.np / p->bb.tm) * B : 0;
    const size_t nbnorm = B > 1 ? (size_t)lzb_chunks(len) * B : 0;
    const size_t need = ((size_t)(m + 2) * vstride + (size_t)B * (4 * m + 1) + 2 * nseg +
                         (size_t)lz_wide_groups(ncplx) + 2 * (2 * ntl + 2 * nseg) + nbdot + nbnorm) * sizeof(double);
    if (need > p->lz_bytes) {
        if (p->lz_mem) (void)hipFree(p->lz_mem);
        p->lz_mem = nullptr;
        p->lz_bytes = 0;
        for (auto it = p->graphs.begin(); it != p->graphs.end();) {  // captured with the old workspace
            if (it->first.rfind("lz:", 0) == 0) {
                (void)hipGraphExecDestroy(it->second);
                it = p->graphs.erase(it);
            } else {
                ++it;
            }
        }
        if (hipMalloc(&p->lz_mem, need) != hipSuccess) {
            (void)hipGetLastError();
            return fail(TDSE_E_NOMEM, "hipMalloc of the Lanczos workspace failed");
        }
        p->lz_bytes = need;
    }
    LzWork w;
    w.V = p->lz_mem;                             // v_1 .. v_m, then w
    w.W = w.V + (size_t)m * vstride;
    w.C = w.W + vstride;
    w.alpha = w.C + vstride;
    w.beta = w.alpha + (size_t)B * m;
    w.beta0 = w.beta + (size_t)B * m;
    w.y = w.beta0 + B;                           // [B][m] complex
    w.dotp = w.y + (size_t)2 * B * m;
    w.normp = w.dotp + nseg;
    {
        double *pp = w.normp + nseg + lz_wide_groups(ncplx);
        for (int q = 0; q < 2; ++q) {
            w.qp[q] = pp;  // two parts per tile
            pp += 2 * ntl;
            w.ep[q] = pp;
            pp += nseg;
            w.np[q] = pp;
            pp += nseg;
        }
        w.bdot = pp;
        pp += nbdot;
        w.bnorm = pp;
    }
    w.vstride = vstride;
    w.len = len;
    w.ncplx = ncplx;
    const int64_t rows = ckpt ? nsteps / K + 1 : 0;
    if (ckpt) TDSE_HIP(lz_ckpt0(c0, ckpt, B, len, rows, s));
    // Single pulse, no checkpoints: whole 64-step chunks replay a captured
    // graph on the plan's state vector (the launches of a step are many and
    // short, so enqueueing them one by one would dominate).
    const bool capture = B == 1 && !ckpt && graphs_enabled() && nsteps >= CHUNK_STEPS;
    double *c = capture ? w.C : cT;
    if (c != c0) TDSE_HIP(hipMemcpyAsync(c, c0, vstride * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (B == 1) {
        CallDesc d{};
        d.nsteps = nsteps;
        d.field = field;
        d.ckpt_every = 1;
        d.dt = dt;
        d.slots = 1;
        TDSE_HIP(set_desc(p->vb.desc, d, s));
    }
    hipGraphExec_t ge = nullptr;
    if (capture) {
        char key[64];
        snprintf(key, sizeof key, "lz:%d:%d", m, CHUNK_STEPS);
        auto it = p->graphs.find(key);
        if (it != p->graphs.end()) {
            ge = it->second;
        } else {
            hipStream_t cs;
            TDSE_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
            // offsets 0 .. 63 of a chunk; field and dt come from the descriptor
            if (e == hipSuccess)
                e = lz_enqueue_steps(p, w, m, dt, &p->vb.desc->dt, nsteps, field, 0, CHUNK_STEPS, 0, w.C, nullptr, K,
                                     0, cs);
            hipError_t e2 = hipStreamEndCapture(cs, &g);
            if (e == hipSuccess) e = e2;
            if (e == hipSuccess) e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
            (void)hipStreamDestroy(cs);
            if (e != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return hip_fail(e, "graph capture of a Lanczos chunk");
            }
            p->graphs[key] = ge;
            p->graph_defs.push_back(g);
        }
    }
    for (int64_t done = 0; done < nsteps; done += CHUNK_STEPS) {
        const int64_t count = nsteps - done < CHUNK_STEPS ? nsteps - done : CHUNK_STEPS;
        if (B == 1) TDSE_HIP(chunk_begin(p->vb.desc, done, s));
        if (ge && count == CHUNK_STEPS) TDSE_HIP(hipGraphLaunch(ge, s));
        else TDSE_HIP(lz_enqueue_steps(p, w, m, dt, nullptr, nsteps, field, done, count, done, c, ckpt, K, rows, s));
    }
    if (c != cT) TDSE_HIP(hipMemcpyAsync(cT, c, vstride * sizeof(double), hipMemcpyDeviceToDevice, s));
    return TDSE_OK;
}

// ---------------------------------------------------------------------------
// Discrete adjoint of the batched RK4 / Taylor map (reverse sweep over
// checkpointed segments; the forward states inside a segment are recomputed
// from its checkpoint and the inputs of every product of a step are kept:
// the four stage inputs of RK4, the terms T_0 .. T_{p-1} of Taylor-p).

static tdse_status adj_workspace(tdse_plan p, int32_t K, int nprod, bool need_ckpt, int64_t nsteps, double **fwd,
                                 double **ustore, double **gpart, double **ickpt) {
    const BatBuffers &b = p->bb;
    const size_t usz = (size_t)(b.lmax + 1) * b.np * b.ldu;
    const int rowtiles = (b.lmax + 1) * (b.np / b.tm);
    const size_t ns = (size_t)(b.lmax + 1) * b.n;
    const size_t n_fwd = 4 * usz, n_us = (size_t)K * nprod * usz, n_gp = (size_t)K * nprod * rowtiles * b.batch;
    const size_t n_ck = need_ckpt ? (size_t)b.batch * (size_t)(nsteps / K + 1) * 2 * ns + (size_t)b.batch * 2 * ns : 0;
    const size_t bytes = (n_fwd + n_us + n_gp + n_ck) * sizeof(double);
    if (bytes > p->adj_bytes) {
        if (p->adj_mem) (void)hipFree(p->adj_mem);
    if (p->ada_mem) (void)hipFree(p->ada_mem);
        p->adj_mem = nullptr;
        p->adj_bytes = 0;
        if (hipMalloc(&p->adj_mem, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return fail(TDSE_E_NOMEM, "hipMalloc of the adjoint workspace failed");
        }
        p->adj_bytes = bytes;
    }
    *fwd = p->adj_mem;
    *ustore = *fwd + n_fwd;
    *gpart = *ustore + n_us;
    *ickpt = need_ckpt ? *gpart + n_gp : nullptr;
    return TDSE_OK;
}

static tdse_status bat_adjoint(tdse_plan p, tdse_method method, int order, double dt, int64_t nsteps,
                               const double *field, const double *c0, const double *ckpt, int32_t K,
                               const double *lambdaT, double *grad, double *lambda0, hipStream_t s) {
    const BatBuffers &pb = p->bb;
    const size_t ns = (size_t)(pb.lmax + 1) * pb.n;
    const size_t usz = (size_t)(pb.lmax + 1) * pb.np * pb.ldu;
    const int rowtiles = (pb.lmax + 1) * (pb.np / pb.tm);
    const int64_t rows = nsteps / K + 1;
    const bool rk4 = method == TDSE_RK4;
    const int nprod = rk4 ? 4 : order, slots = rk4 ? 3 : 1;
    double *fwd, *ustore, *gpart, *ickpt;
    tdse_status st = adj_workspace(p, K, nprod, ckpt == nullptr, nsteps, &fwd, &ustore, &gpart, &ickpt);
    if (st != TDSE_OK) return st;
    if (!ckpt) {
        // forward pass writing checkpoints into the workspace (c(T) goes to its tail)
        double *cT = ickpt + (size_t)pb.batch * rows * 2 * ns;
        st = bat_propagate(p, method, order, dt, nsteps, field, c0, cT, ickpt, K, s);
        if (st != TDSE_OK) return st;
        ckpt = ickpt;
    }
    // forward-recompute view: same Hamiltonian, its own state buffers
    BatBuffers fb = pb;
    fb.field = field;
    fb.u[0] = fwd;
    fb.u[1] = fwd + usz;
    fb.c = fwd + 2 * usz;
    fb.acc = fwd + 3 * usz;
    // adjoint state: c = lambda, acc = co-state sum, u = product input (RK4:
    // kbar of the stage; Taylor: (dt/m) Tbar_m)
    BatBuffers ab = pb;
    ab.field = field;
    TDSE_HIP(bat_pack_strided(ab, lambdaT, 2 * ns, rk4 ? dt / 6.0 : dt / order, s));
    int apar = 0;
    std::vector<BatLaunch> fsched;
    bat_schedule(method, order, fsched);
    const int64_t nseg = (nsteps + K - 1) / K;
    for (int64_t sg = nseg - 1; sg >= 0; --sg) {
        const int64_t k0 = sg * K, len = nsteps - k0 < K ? nsteps - k0 : K;
        TDSE_HIP(bat_pack_strided(fb, ckpt + (size_t)sg * 2 * ns, (size_t)rows * 2 * ns, 1.0, s));
        int fpar = 0;
        for (int64_t k = k0; k < k0 + len; ++k) {
            for (int j = 0; j < nprod; ++j) {
                BatLaunch L = fsched[j];
                L.parity = fpar;
                L.dt = dt;
                L.step = k;
                L.nsteps = nsteps;
                L.slots = slots;
                L.ustore = ustore + ((size_t)(k - k0) * nprod + j) * usz;
                TDSE_HIP(bat_launch_stage(fb, L, s));
                fpar ^= 1;
            }
        }
        for (int64_t k = k0 + len - 1; k >= k0 && !rk4; --k) {
            // Taylor term m = p..1: input (dt/m) Tbar_m gives ubar = (i dt/m) H Tbar_m,
            // Tbar_{m-1} = lambda + ubar; the next input is (dt/(m-1)) Tbar_{m-1},
            // and after m = 1 the new lambda Tbar_0 scaled by dt/p.
            for (int m = order; m >= 1; --m) {
                BatLaunch L{};
                L.kind = m > 1 ? CK_ADJ_MID : CK_ADJ_LAST;
                L.slot = 0;
                L.first = 1;
                L.parity = apar;
                L.dt = dt;
                L.step = k;
                L.nsteps = nsteps;
                L.slots = 1;
                L.ustore = ustore + ((size_t)(k - k0) * nprod + (m - 1)) * usz;
                L.gpart = gpart + ((size_t)(k - k0) * nprod + (m - 1)) * rowtiles * pb.batch;
                L.p_lam = m > 1 ? dt / (m - 1) : dt / order;
                L.p_ub = m > 1 ? dt / (m - 1) : 0.0;
                TDSE_HIP(bat_launch_adjoint(ab, L, s));
                apar ^= 1;
            }
        }
        for (int64_t k = k0 + len - 1; k >= k0 && rk4; --k) {
            for (int j = 4; j >= 1; --j) {
                BatLaunch L{};
                L.kind = j > 1 ? CK_ADJ_MID : CK_ADJ_LAST;
                L.slot = j == 4 ? 2 : (j == 1 ? 0 : 1);
                L.first = j == 4 ? 1 : 0;
                L.parity = apar;
                L.dt = dt;
                L.step = k;
                L.nsteps = nsteps;
                L.slots = 3;
                L.ustore = ustore + ((size_t)(k - k0) * 4 + (j - 1)) * usz;
                L.gpart = gpart + ((size_t)(k - k0) * 4 + (j - 1)) * rowtiles * pb.batch;
                // next co-state input: kbar_{j-1} = b_{j-1} dt lambda + alpha_j dt ubar_j
                if (j == 4) { L.p_lam = dt / 3.0; L.p_ub = dt; }
                else if (j == 3) { L.p_lam = dt / 3.0; L.p_ub = dt / 2.0; }
                else if (j == 2) { L.p_lam = dt / 6.0; L.p_ub = dt / 2.0; }
                else { L.p_lam = dt / 6.0; L.p_ub = 0.0; }
                TDSE_HIP(bat_launch_adjoint(ab, L, s));
                apar ^= 1;
            }
        }
        TDSE_HIP(bat_reduce_grad(gpart, rowtiles, pb.batch, k0, len, nsteps, nprod, rk4 ? 1 : 0, grad, s));
    }
    if (lambda0) TDSE_HIP(bat_unpack(ab, lambda0, s));
    return TDSE_OK;
}

// A batched (matrix-core) plan of batch 1 over the same Hamiltonian, built
// from a single-vector plan's device copies; used for that plan's adjoint.
static tdse_status create_batched_twin(tdse_plan p, hipStream_t s) {
    tdse_plan q = new (std::nothrow) tdse_plan_s();
    if (!q) return fail(TDSE_E_NOMEM, "host allocation failed");
    q->lmax = p->lmax;
    q->n = p->n;
    q->batch = 1;
    q->gauge = p->gauge;
    q->device = p->device;
    double *rowmajor = nullptr;
    if (p->lmax > 0) {
        if (hipMalloc(&rowmajor, (size_t)p->lmax * p->n * p->n * sizeof(double)) != hipSuccess) {
            (void)hipGetLastError();
            delete q;
            return fail(TDSE_E_NOMEM, "hipMalloc for the adjoint twin plan failed");
        }
        hipError_t e = vec_untile(p->dip, rowmajor, p->lmax, p->n, p->T, s);
        if (e != hipSuccess) {
            (void)hipFree(rowmajor);
            delete q;
            return hip_fail(e, "untile of the dipole");
        }
    }
    tdse_status st = bat_create(q, p->en, rowmajor, s, nullptr);
    if (rowmajor) (void)hipFree(rowmajor);
    if (st != TDSE_OK) {
        std::string msg = g_last_error;
        tdse_destroy(q);
        return fail(st, msg);
    }
    p->adj_plan = q;
    return TDSE_OK;
}

// Runge-Kutta-Fehlberg runs on the batched kernels; a batch-1 plan uses its
// batched twin (built on first use, shared with the adjoint).
static tdse_status rkf_propagate(tdse_plan p, double dt, int64_t nsteps, const double *field, const double *c0,
                                 double *cT, double *err, double *ckpt, int32_t K, hipStream_t s) {
    tdse_plan q = p;
    if (p->batch == 1) {
        if (!p->adj_plan) {
            tdse_status st = create_batched_twin(p, s);
            if (st != TDSE_OK) return st;
        }
        q = p->adj_plan;
    }
    return bat_propagate(q, TDSE_RKF45, 0, dt, nsteps, field, c0, cT, ckpt, K, s, err);
}

}  // namespace tdse

using namespace tdse;

extern "C" {

int tdse_abi_version(void) { return TDSE_ABI_VERSION; }

const char *tdse_last_error(void) { return g_last_error.c_str(); }

tdse_status tdse_create(tdse_plan *out, const double *energies, const double *dipole,
                        int32_t lmax, int32_t n, int32_t batch, void *stream) {
    return tdse_create_gauge(out, energies, dipole, TDSE_LENGTH, lmax, n, batch, stream);
}

tdse_status tdse_create_gauge(tdse_plan *out, const double *energies, const double *coupling, tdse_gauge gauge,
                              int32_t lmax, int32_t n, int32_t batch, void *stream) {
    clear_error();
    std::string why;
    tdse_status st = validate_create(out, energies, coupling, lmax, n, batch, &why);
    if (st != TDSE_OK) return fail(st, why);
    if (gauge != TDSE_LENGTH && gauge != TDSE_VELOCITY) return fail(TDSE_E_INVAL, "unknown gauge");
    return create_plan(out, energies, coupling, (int32_t)gauge, lmax, n, batch,
                       reinterpret_cast<hipStream_t>(stream), nullptr);
}

}  // extern "C"

namespace tdse {

tdse_status create_plan(tdse_plan *out, const double *energies, const double *dipole, int32_t gauge, int32_t lmax,
                        int32_t n, int32_t batch, hipStream_t s, const TileChoice *force) {
    tdse_status st;
    tdse_plan p = new (std::nothrow) tdse_plan_s();
    if (!p) return fail(TDSE_E_NOMEM, "host allocation failed");
    p->gauge = gauge;
    p->lmax = lmax;
    p->n = n;
    p->batch = batch;
    TDSE_HIP(hipGetDevice(&p->device));
    if (batch > 1) {
        st = bat_create(p, energies, dipole, s, force);
        if (st != TDSE_OK) {
            std::string msg = g_last_error;
            tdse_destroy(p);
            return fail(st, msg);
        }
        *out = p;
        return TDSE_OK;
    }
    p->ld = VEC_TILE_MAX;
    p->T = (n + VEC_TILE_MAX - 1) / VEC_TILE_MAX;
    {
        TileChoice tc{0, 0, 0, 0, 0};
        if (force) tc = *force;
        else tune_lookup(lmax, n, 1, &tc);
        if (tc.T >= p->T && tc.T <= (n + 15) / 16) p->T = tc.T;  // segments of whole 16-row units
        // a forced tile count selects the tiled kernels even for small problems
        p->small = tc.T == 0 && small_eligible(lmax, n);
    }
    // Beyond two tile workgroups per CU the product launches stream the dipole
    // from HBM, and re-reading every segment's partials in each of its T
    // tiles would add (T + 3) / 64 of the dipole traffic: completion then runs
    // once per segment in a launch of its own. $TDSE_SPLIT=0/1 overrides.
    p->split = (int64_t)lmax * p->T * p->T > 512;
    if (const char *sp = getenv("TDSE_SPLIT")) {
        if (sp[0] == '0') p->split = false;
        if (sp[0] == '1') p->split = true;
    }
    if (p->T > 16) {
        delete p;
        return fail(TDSE_E_UNSUPPORTED, "n > 2048 states per partial wave is not supported");
    }
    const size_t ns = (size_t)(lmax + 1) * n;
    const size_t dip_elems = (size_t)lmax * n * n;
    const size_t tiled_elems = (size_t)lmax * p->T * p->T * VEC_TILE_MAX * VEC_TILE_MAX;
    double *stage = nullptr;
    hipError_t e = hipMalloc(&p->en, ns * sizeof(double));
    if (e == hipSuccess && lmax > 0) e = hipMalloc(&p->dip, tiled_elems * sizeof(double));
    if (e == hipSuccess && lmax > 0) e = hipMalloc(&stage, dip_elems * sizeof(double));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        if (stage) (void)hipFree(stage);
        tdse_destroy(p);
        return fail(TDSE_E_NOMEM, "hipMalloc of the Hamiltonian failed");
    }
    e = hipMemcpyAsync(p->en, energies, ns * sizeof(double), hipMemcpyDefault, s);
    if (e == hipSuccess && lmax > 0)
        e = hipMemcpyAsync(stage, dipole, dip_elems * sizeof(double), hipMemcpyDefault, s);
    if (e == hipSuccess && lmax > 0) e = vec_layout(stage, p->dip, lmax, n, p->T, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    st = e == hipSuccess ? coupling_bounds(p, p->en, stage, s) : TDSE_OK;
    if (stage) (void)hipFree(stage);
    if (e != hipSuccess) {
        tdse_destroy(p);
        return hip_fail(e, "copy of the Hamiltonian into the plan");
    }
    if (st != TDSE_OK) {
        std::string msg = g_last_error;
        tdse_destroy(p);
        return fail(st, msg);
    }
    st = vec_alloc(p);
    if (st != TDSE_OK) {
        std::string msg = g_last_error;
        tdse_destroy(p);
        return fail(st, msg);
    }
    *out = p;
    return TDSE_OK;
}

}  // namespace tdse

extern "C" {

tdse_status tdse_destroy(tdse_plan p) {
    clear_error();
    if (!p) return TDSE_OK;
    (void)hipDeviceSynchronize();
    for (auto &kv : p->graphs) (void)hipGraphExecDestroy(kv.second);
    for (hipGraph_t g : p->graph_defs) (void)hipGraphDestroy(g);
    if (p->scratch) (void)hipFree(p->scratch);
    if (p->bat_mem) (void)hipFree(p->bat_mem);
    if (p->rkf_mem) (void)hipFree(p->rkf_mem);
    if (p->lz_mem) (void)hipFree(p->lz_mem);
    if (p->adj_mem) (void)hipFree(p->adj_mem);
    if (p->adj_plan) tdse_destroy(p->adj_plan);
    if (p->dip) (void)hipFree(p->dip);
    if (p->en) (void)hipFree(p->en);
    delete p;
    return TDSE_OK;
}

tdse_status tdse_plan_shape(tdse_plan p, int32_t *lmax, int32_t *n, int32_t *batch) {
    clear_error();
    if (!p) return fail(TDSE_E_INVAL, "plan is NULL");
    if (lmax) *lmax = p->lmax;
    if (n) *n = p->n;
    if (batch) *batch = p->batch;
    return TDSE_OK;
}

tdse_status tdse_hmul(tdse_plan p, const double *fields, const double *u, double *y, void *stream) {
    clear_error();
    if (!p) return fail(TDSE_E_INVAL, "plan is NULL");
    tdse_status st;
    if ((st = check_dev(fields, "fields")) || (st = check_dev(u, "u")) || (st = check_dev(y, "y")))
        return st;
    if (u == y) return fail(TDSE_E_INVAL, "u and y must not alias");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (p->batch > 1) return bat_hmul(p, fields, u, y, s);
    CallDesc d{};
    d.nsteps = 1;
    d.field = fields;
    d.ckpt_every = 1;
    d.dt = 1.0;
    d.slots = 1;
    TDSE_HIP(set_desc(p->vb.desc, d, s));
    TDSE_HIP(chunk_begin(p->vb.desc, 0, s));
    TDSE_HIP(vec_launch_start(p->vb, 0, u, TDSE_RK4, s));
    VecLaunch L{};
    L.comp = {CK_RK4_END, 0, -1, 0, 1.0 / 6.0, 0.0};
    L.parity = 0;
    L.slots = 1;
    if (p->lmax > 0) TDSE_HIP(vec_launch_tiles(p->vb, L, s));
    else TDSE_HIP(vec_launch_combine(p->vb, L, s));
    VecLaunch H{};
    H.comp = {CK_HMUL, 0, 0, 0, 0.0, 0.0};
    H.parity = 1;
    H.slots = 1;
    H.out = y;
    TDSE_HIP(vec_launch_combine(p->vb, H, s));
    return TDSE_OK;
}

tdse_status tdse_propagate(tdse_plan p, tdse_method method, int32_t order, double dt,
                           int64_t nsteps, const double *field, const double *c0, double *cT,
                           double *ckpt, int32_t ckpt_every, void *stream) {
    clear_error();
    std::string why;
    tdse_status st = validate_propagate(p != nullptr, (int)method, order, dt, nsteps, ckpt != nullptr,
                                        ckpt_every, &why);
    if (st != TDSE_OK) return fail(st, why);
    if (nsteps > 0 && (st = check_dev(field, "field"))) return st;
    if ((st = check_dev(c0, "c0")) || (st = check_dev(cT, "cT"))) return st;
    if (ckpt && (st = check_dev(ckpt, "ckpt"))) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (method == TDSE_LANCZOS) return lz_propagate(p, order, dt, nsteps, field, c0, cT, ckpt, ckpt_every, s);
    if (method == TDSE_RKF45) return rkf_propagate(p, dt, nsteps, field, c0, cT, nullptr, ckpt, ckpt_every, s);
    if (p->batch > 1)
        return bat_propagate(p, method, method == TDSE_RK4 ? 4 : order, dt, nsteps, field, c0, cT, ckpt,
                             ckpt_every, s);
    return vec_propagate(p, method, method == TDSE_RK4 ? 4 : order, dt, nsteps, field, c0, cT, ckpt,
                         ckpt_every, s);
}

tdse_status tdse_adjoint(tdse_plan p, tdse_method method, int32_t order, double dt, int64_t nsteps,
                         const double *field, const double *c0, const double *ckpt,
                         int32_t ckpt_every, const double *lambdaT, double *grad_field,
                         double *lambda0, void *stream) {
    clear_error();
    std::string why;
    tdse_status st = validate_propagate(p != nullptr, (int)method, method == TDSE_TAYLOR ? order : 4, dt, nsteps,
                                        true, ckpt_every, &why);
    if (st != TDSE_OK) return fail(st, why);
    if (method == TDSE_LANCZOS || method == TDSE_RKF45)
        return fail(TDSE_E_UNSUPPORTED, "the adjoint covers RK4 and Taylor-p");
    if (nsteps > 0 && (st = check_dev(field, "field"))) return st;
    if ((st = check_dev(c0, "c0")) || (st = check_dev(lambdaT, "lambdaT"))) return st;
    if (nsteps > 0 && (st = check_dev(grad_field, "grad_field"))) return st;
    if (ckpt && (st = check_dev(ckpt, "ckpt"))) return st;
    if (lambda0 && (st = check_dev(lambda0, "lambda0"))) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    tdse_plan q = p;
    if (p->batch == 1) {
        // batch-1 plans run the adjoint on a batched twin of themselves
        if (!p->adj_plan) {
            st = create_batched_twin(p, s);
            if (st != TDSE_OK) return st;
        }
        q = p->adj_plan;
    }
    return bat_adjoint(q, method, order, dt, nsteps, field, c0, ckpt, ckpt_every, lambdaT, grad_field, lambda0, s);
}

tdse_status tdse_propagate_rkf45(tdse_plan p, double dt, int64_t nsteps, const double *field, const double *c0,
                                 double *cT, double *err, double *ckpt, int32_t ckpt_every, void *stream) {
    clear_error();
    std::string why;
    tdse_status st = validate_propagate(p != nullptr, TDSE_RKF45, 0, dt, nsteps, ckpt != nullptr, ckpt_every, &why);
    if (st != TDSE_OK) return fail(st, why);
    if (nsteps > 0 && (st = check_dev(field, "field"))) return st;
    if ((st = check_dev(c0, "c0")) || (st = check_dev(cT, "cT"))) return st;
    if (ckpt && (st = check_dev(ckpt, "ckpt"))) return st;
    if (err && nsteps > 0 && (st = check_dev(err, "err"))) return st;
    return rkf_propagate(p, dt, nsteps, field, c0, cT, err, ckpt, ckpt_every, reinterpret_cast<hipStream_t>(stream));
}

tdse_status tdse_check_stability(tdse_plan p, tdse_method method, int32_t order, double dt, double fmax,
                                 double *theta, double *bound) {
    clear_error();
    std::string why;
    tdse_status st = validate_propagate(p != nullptr, (int)method, method == TDSE_RK4 || method == TDSE_RKF45 ? 1 : order,
                                        dt, 0, false, 0, &why);
    if (st != TDSE_OK) return fail(st, why);
    if (!isfinite(fmax)) return fail(TDSE_E_INVAL, "fmax must be finite");
    double th = 0.0, bd = 0.0;
    st = check_stability(method, order, dt, p->emax, fmax, p->dnorm, &th, &bd);
    if (theta) *theta = th;
    if (bound) *bound = bd;
    if (st != TDSE_OK) {
        char buf[240];
        snprintf(buf, sizeof buf,
                 "unstable step: dt (max|E| + |F| ||D||) = %.6g exceeds the method's imaginary-axis bound %.6g "
                 "(max|E| = %.6g, ||D|| <= %.6g)",
                 th, bd, p->emax, p->dnorm);
        return fail(TDSE_E_UNSTABLE, buf);
    }
    return TDSE_OK;
}

tdse_status tdse_propagate_adaptive(tdse_plan p, double t_final, double dt0, double tol, double dt_min,
                                    int64_t max_steps, tdse_field_fn field_fn, void *ctx, const double *c0,
                                    double *cT, double *steps, int64_t *nsteps_taken, void *stream) {
    clear_error();
    if (!p) return fail(TDSE_E_INVAL, "plan is NULL");
    if (!field_fn) return fail(TDSE_E_INVAL, "field_fn is NULL");
    if (!nsteps_taken) return fail(TDSE_E_INVAL, "nsteps_taken is NULL");
    if (!(t_final >= 0.0) || !isfinite(t_final)) return fail(TDSE_E_INVAL, "t_final must be finite and >= 0");
    if (!(dt0 > 0.0) || !isfinite(dt0)) return fail(TDSE_E_INVAL, "dt0 must be finite and > 0");
    if (!(dt_min > 0.0) || !isfinite(dt_min)) return fail(TDSE_E_INVAL, "dt_min must be finite and > 0");
    if (!(tol > 0.0) || !isfinite(tol)) return fail(TDSE_E_INVAL, "tol must be finite and > 0");
    if (max_steps < 0) return fail(TDSE_E_INVAL, "max_steps must be >= 0");
    tdse_status st;
    if ((st = check_dev(c0, "c0")) || (st = check_dev(cT, "cT"))) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int B = p->batch;
    const size_t len = (size_t)B * 2 * (p->lmax + 1) * p->n;
    const size_t need = ((size_t)B * 6 + 2 * len + (size_t)B) * sizeof(double);
    if (need > p->ada_bytes) {
        if (p->ada_mem) (void)hipFree(p->ada_mem);
        p->ada_mem = nullptr;
        p->ada_bytes = 0;
        if (hipMalloc(&p->ada_mem, need) != hipSuccess) {
            (void)hipGetLastError();
            return fail(TDSE_E_NOMEM, "hipMalloc of the adaptive-step workspace failed");
        }
        p->ada_bytes = need;
    }
    double *dfield = p->ada_mem, *cur = dfield + (size_t)B * 6, *nxt = cur + len, *derr = nxt + len;
    std::vector<double> hfield((size_t)B * 6), herr(B);
    TDSE_HIP(hipMemcpyAsync(cur, c0, len * sizeof(double), hipMemcpyDeviceToDevice, s));
    double t = 0.0, dt = dt0;
    int64_t taken = 0, tried = 0;
    while (t < t_final * (1.0 - 1e-14) && tried < max_steps) {
        const double h = dt < t_final - t ? dt : t_final - t;
        field_fn(t, h, hfield.data(), ctx);
        TDSE_HIP(hipMemcpyAsync(dfield, hfield.data(), hfield.size() * sizeof(double), hipMemcpyHostToDevice, s));
        TDSE_HIP_ST(rkf_propagate(p, h, 1, dfield, cur, nxt, derr, nullptr, 1, s));
        TDSE_HIP(hipMemcpyAsync(herr.data(), derr, B * sizeof(double), hipMemcpyDeviceToHost, s));
        TDSE_HIP(hipStreamSynchronize(s));
        double e = 0.0;
        for (int b = 0; b < B; ++b) e = herr[b] > e ? herr[b] : e;
        ++tried;
        if (e <= tol || h <= dt_min) {
            std::swap(cur, nxt);
            t += h;
            if (steps) steps[taken] = h;
            ++taken;
        }
        const double fac = e == 0.0 ? 2.0 : std::min(2.0, std::max(0.2, 0.9 * pow(tol / e, 0.2)));
        dt = std::max(dt_min, h * fac);
    }
    TDSE_HIP(hipMemcpyAsync(cT, cur, len * sizeof(double), hipMemcpyDeviceToDevice, s));
    TDSE_HIP(hipStreamSynchronize(s));
    *nsteps_taken = taken;
    if (t < t_final * (1.0 - 1e-14)) return fail(TDSE_E_INVAL, "max_steps reached before t_final");
    return TDSE_OK;
}

// Tile count a group member streams with: the default ceil(n / 128).
static int group_tiles(int n) { return (n + VEC_TILE_MAX - 1) / VEC_TILE_MAX; }

// Captured group chunks hold the work-list addresses: drop them before the
// lists move.
static void drop_group_graphs(tdse_group g) {
    if (g->graphs.empty() && g->graph_defs.empty()) return;
    (void)hipDeviceSynchronize();
    for (auto &kv : g->graphs) (void)hipGraphExecDestroy(kv.second);
    for (hipGraph_t gd : g->graph_defs) (void)hipGraphDestroy(gd);
    g->graphs.clear();
    g->graph_defs.clear();
}

tdse_status tdse_group_create(tdse_group *out, int32_t count, const tdse_plan *plans, void *stream) {
    clear_error();
    (void)stream;
    if (!out) return fail(TDSE_E_INVAL, "out is NULL");
    if (count < 1) return fail(TDSE_E_INVAL, "count must be >= 1");
    if (!plans) return fail(TDSE_E_INVAL, "plans is NULL");
    for (int32_t k = 0; k < count; ++k) {
        const tdse_plan p = plans[k];
        if (!p) return fail(TDSE_E_INVAL, "plans[" + std::to_string(k) + "] is NULL");
        if (p->batch != 1) return fail(TDSE_E_INVAL, "group members must be batch-1 plans");
        if (group_tiles(p->n) > 8)
            return fail(TDSE_E_UNSUPPORTED, "group members need n <= 1024 (plans[" + std::to_string(k) +
                                                "] has n = " + std::to_string(p->n) + ")");
        if (p->device != plans[0]->device) return fail(TDSE_E_INVAL, "group members must share one device");
        for (int32_t m = 0; m < k; ++m)
            if (plans[m] == p)  // one plan's state buffers cannot hold two instances
                return fail(TDSE_E_INVAL, "plans[" + std::to_string(m) + "] and plans[" + std::to_string(k) +
                                              "] are the same plan");
    }
    tdse_group g = new (std::nothrow) tdse_group_s();
    if (!g) return fail(TDSE_E_NOMEM, "host allocation failed");
    g->plans.assign(plans, plans + count);
    g->retiled.assign(count, nullptr);
    // A member built with more tiles than the default (a tuned or forced
    // count) streams a copy of its blocks at the default count: inside a group
    // every CU already has work, so the extra workgroups smaller tiles buy a
    // lone plan do not help, while each of its patches streams fewer bytes
    // per workgroup (measured: a group on the lone-tuned counts ran at 0.98x).
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    double *rowmajor = nullptr;
    size_t row_cap = 0;
    hipError_t e = hipSuccess;
    for (int32_t k = 0; k < count && e == hipSuccess; ++k) {
        const tdse_plan p = plans[k];
        const int t0 = group_tiles(p->n);
        if (p->lmax == 0 || p->T == t0) continue;
        const size_t dense = (size_t)p->lmax * p->n * p->n;
        if (dense > row_cap) {
            if (rowmajor) (void)hipFree(rowmajor);
            rowmajor = nullptr;
            row_cap = 0;
            if ((e = hipMalloc(&rowmajor, dense * sizeof(double))) != hipSuccess) break;
            row_cap = dense;
        }
        const size_t tiled = (size_t)p->lmax * t0 * t0 * VEC_TILE_MAX * VEC_TILE_MAX;
        if ((e = hipMalloc(&g->retiled[k], tiled * sizeof(double))) != hipSuccess) break;
        e = vec_untile(p->dip, rowmajor, p->lmax, p->n, p->T, s);
        if (e == hipSuccess) e = vec_layout(rowmajor, g->retiled[k], p->lmax, p->n, t0, s);
        // the next member reuses the row-major buffer
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    if (rowmajor) (void)hipFree(rowmajor);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        tdse_group_destroy(g);
        return e == hipErrorOutOfMemory ? fail(TDSE_E_NOMEM, "hipMalloc of a re-tiled group member failed")
                                        : hip_fail(e, "re-tiling of a group member");
    }
    *out = g;
    return TDSE_OK;
}

tdse_status tdse_group_propagate(tdse_group g, tdse_method method, int32_t order, double dt,
                                 const int64_t *nsteps, const double *const *fields,
                                 const double *const *c0, double *const *cT, void *stream) {
    clear_error();
    (void)order;
    if (!g) return fail(TDSE_E_INVAL, "group is NULL");
    if (method != TDSE_RK4 && method != TDSE_TAYLOR) return fail(TDSE_E_INVAL, "unknown method");
    if (method != TDSE_RK4) return fail(TDSE_E_UNSUPPORTED, "groups propagate with RK4 only");
    if (!(dt > 0.0) || !isfinite(dt)) return fail(TDSE_E_INVAL, "dt must be finite and > 0");
    if (!nsteps || !fields || !c0 || !cT) return fail(TDSE_E_INVAL, "nsteps, fields, c0 and cT must not be NULL");
    const int count = (int)g->plans.size();
    tdse_status st;
    for (int k = 0; k < count; ++k) {
        if (nsteps[k] < 0) return fail(TDSE_E_INVAL, "nsteps[" + std::to_string(k) + "] < 0");
        if (nsteps[k] > 0 && (st = check_dev(fields[k], "fields[k]"))) return st;
        if ((st = check_dev(c0[k], "c0[k]")) || (st = check_dev(cT[k], "cT[k]"))) return st;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // Instances without dipole blocks run on their own; the others are
    // ordered by step count (descending) so the active set of every round is
    // a prefix of the work list.
    std::vector<int> order_idx;
    for (int k = 0; k < count; ++k) {
        if (g->plans[k]->lmax == 0)
            TDSE_HIP_ST(tdse_propagate(g->plans[k], TDSE_RK4, 0, dt, nsteps[k], fields[k], c0[k], cT[k], nullptr,
                                       0, stream));
        else
            order_idx.push_back(k);
    }
    std::stable_sort(order_idx.begin(), order_idx.end(), [&](int a, int b) { return nsteps[a] > nsteps[b]; });
    g->tiles.clear();
    g->segs.clear();
    g->insts.clear();
    std::vector<int64_t> prefix(1, 0), seg_prefix(1, 0);
    for (size_t q = 0; q < order_idx.size(); ++q) {
        const tdse_plan p = g->plans[order_idx[q]];
        GroupInst gi{};
        gi.b = p->vb;
        if (g->retiled[order_idx[q]]) {
            // the default tile count over the plan's own state and partial
            // buffers (sized for its larger count)
            gi.b.dip = g->retiled[order_idx[q]];
            gi.b.T = group_tiles(p->n);
        }
        gi.field = fields[order_idx[q]];
        gi.nsteps = nsteps[order_idx[q]];
        g->insts.push_back(gi);
        const int T = gi.b.T;
        const int npd = patch_np(T);  // patches per block dimension
        for (int l = 0; l < p->lmax; ++l)
            for (int i = 0; i < npd; ++i)
                for (int j = 0; j < npd; ++j) g->tiles.push_back({(int32_t)q, (int16_t)l, (int8_t)i, (int8_t)j});
        for (int mm = 0; mm <= p->lmax; ++mm)
            for (int qq = 0; qq < T; ++qq) g->segs.push_back({(int32_t)q, (int16_t)mm, (int16_t)qq});
        prefix.push_back((int64_t)g->tiles.size());
        seg_prefix.push_back((int64_t)g->segs.size());
    }
    if (order_idx.empty()) return TDSE_OK;
    if (g->tiles.size() > g->tiles_cap) {
        drop_group_graphs(g);
        if (g->d_tiles) (void)hipFree(g->d_tiles);
        g->d_tiles = nullptr;
        g->tiles_cap = 0;
        if (hipMalloc(&g->d_tiles, g->tiles.size() * sizeof(GroupTile)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(TDSE_E_NOMEM, "hipMalloc of the group work list failed");
        }
        g->tiles_cap = g->tiles.size();
    }
    if (g->segs.size() > g->segs_cap) {
        drop_group_graphs(g);
        if (g->d_segs) (void)hipFree(g->d_segs);
        g->d_segs = nullptr;
        g->segs_cap = 0;
        if (hipMalloc(&g->d_segs, g->segs.size() * sizeof(GroupSeg)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(TDSE_E_NOMEM, "hipMalloc of the group segment list failed");
        }
        g->segs_cap = g->segs.size();
    }
    if (g->insts.size() > g->insts_cap) {
        drop_group_graphs(g);
        if (g->d_insts) (void)hipFree(g->d_insts);
        g->d_insts = nullptr;
        g->insts_cap = 0;
        if (hipMalloc(&g->d_insts, g->insts.size() * sizeof(GroupInst)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(TDSE_E_NOMEM, "hipMalloc of the group instance table failed");
        }
        g->insts_cap = g->insts.size();
    }
    TDSE_HIP(hipMemcpyAsync(g->d_tiles, g->tiles.data(), g->tiles.size() * sizeof(GroupTile),
                            hipMemcpyHostToDevice, s));
    TDSE_HIP(hipMemcpyAsync(g->d_segs, g->segs.data(), g->segs.size() * sizeof(GroupSeg),
                            hipMemcpyHostToDevice, s));
    TDSE_HIP(hipMemcpyAsync(g->d_insts, g->insts.data(), g->insts.size() * sizeof(GroupInst),
                            hipMemcpyHostToDevice, s));
    if (!g->d_desc && hipMalloc(&g->d_desc, sizeof(GroupDesc)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(TDSE_E_NOMEM, "hipMalloc of the group descriptor failed");
    }
    for (size_t q = 0; q < order_idx.size(); ++q)
        TDSE_HIP(vec_launch_start(g->insts[q].b, 0, c0[order_idx[q]], TDSE_RK4, s));
    // Rounds go in chunks of GROUP_CHUNK_ROUNDS; a chunk's launches cover the
    // instances active at its first round (the kernels skip instances that
    // finish inside the chunk). Whole chunks replay a captured graph.
    const int64_t rounds = 4 * nsteps[order_idx[0]];
    size_t active = order_idx.size();
    for (int64_t r = 0; r < rounds; r += GROUP_CHUNK_ROUNDS) {
        while (active > 0 && 4 * nsteps[order_idx[active - 1]] <= r) --active;
        const int nt = (int)prefix[active], ns = (int)seg_prefix[active];
        const int len = (int)std::min<int64_t>(GROUP_CHUNK_ROUNDS, rounds - r);
        TDSE_HIP(group_set_desc(g->d_desc, r, dt, s));
        hipGraphExec_t ge = nullptr;
        if (graphs_enabled() && len == GROUP_CHUNK_ROUNDS) {
            const int64_t key = ((int64_t)nt << 32) | (uint32_t)ns;  // what a capture depends on
            auto it = g->graphs.find(key);
            if (it != g->graphs.end()) {
                ge = it->second;
            } else {
                hipStream_t cs;
                TDSE_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
                hipGraph_t gd = nullptr;
                hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
                for (int off = 0; e == hipSuccess && off < GROUP_CHUNK_ROUNDS; ++off)
                    e = group_launch_round(g->d_segs, ns, g->d_tiles, nt, g->d_insts, g->d_desc, off, cs);
                hipError_t e2 = hipStreamEndCapture(cs, &gd);
                if (e == hipSuccess) e = e2;
                if (e == hipSuccess) e = hipGraphInstantiate(&ge, gd, nullptr, nullptr, 0);
                (void)hipStreamDestroy(cs);
                if (e != hipSuccess) {
                    if (gd) (void)hipGraphDestroy(gd);
                    return hip_fail(e, "graph capture of a group chunk");
                }
                g->graphs[key] = ge;
                g->graph_defs.push_back(gd);
            }
            TDSE_HIP(hipGraphLaunch(ge, s));
        } else {
            for (int off = 0; off < len; ++off)
                TDSE_HIP(group_launch_round(g->d_segs, ns, g->d_tiles, nt, g->d_insts, g->d_desc, off, s));
        }
    }
    // final completion of every instance (c(T) -> cT), over the partials of
    // the group's rounds (the instance table's tile count)
    for (size_t q = 0; q < order_idx.size(); ++q) {
        const int k = order_idx[q];
        const VecBuffers &vb = g->insts[q].b;
        CallDesc d{};
        d.nsteps = nsteps[k];
        d.field = fields[k];
        d.ckpt_every = 1;
        d.dt = dt;
        d.slots = 3;
        TDSE_HIP(set_desc(vb.desc, d, s));
        const int64_t base = nsteps[k] > 0 ? ((nsteps[k] - 1) / CHUNK_STEPS) * CHUNK_STEPS : 0;
        TDSE_HIP(chunk_begin(vb.desc, base, s));
        VecLaunch L{};
        L.comp = final_completion(TDSE_RK4, 4);
        L.off = (int32_t)(nsteps[k] - base);
        L.parity = 0;
        L.finish = 1;
        L.slots = 3;
        L.np = patch_np(vb.T);  // the group's products rounds are patch launches
        L.out = cT[k];
        TDSE_HIP(vec_launch_combine(vb, L, s));
    }
    return TDSE_OK;
}

tdse_status tdse_group_destroy(tdse_group g) {
    clear_error();
    if (!g) return TDSE_OK;
    (void)hipDeviceSynchronize();
    if (g->d_tiles) (void)hipFree(g->d_tiles);
    drop_group_graphs(g);
    if (g->d_segs) (void)hipFree(g->d_segs);
    if (g->d_insts) (void)hipFree(g->d_insts);
    if (g->d_desc) (void)hipFree(g->d_desc);
    for (double *r : g->retiled)
        if (r) (void)hipFree(r);
    delete g;
    return TDSE_OK;
}

}  // extern "C"
