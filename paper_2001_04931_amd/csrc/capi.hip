// C ABI of libempc.so: argument validation, dispatch and the solve loop.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "internal.hpp"

using namespace empc;

namespace {

thread_local char g_err[512] = "";

empc_status fail(empc_status s, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return s;
}

empc_status device_status(hipError_t e, const char *where) {
    if (e == hipSuccess) return EMPC_OK;
    return fail(EMPC_EDEVICE, "%s: %s", where, hipGetErrorString(e));
}

// An asynchronous fault of earlier work is reported by the next call.
empc_status check_prior() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(EMPC_EDEVICE, "earlier device error: %s", hipGetErrorString(e));
    return EMPC_OK;
}

size_t esize(const empc_problem *P) { return P->dtype == EMPC_F64 ? 8 : 4; }

empc_status validate_problem(const empc_problem *P) {
    if (!P) return fail(EMPC_EINVAL, "problem is NULL");
    if (P->dtype != EMPC_F32 && P->dtype != EMPC_F64)
        return fail(EMPC_EINVAL, "unknown dtype %d", P->dtype);
    if (P->model != EMPC_LINEAR && P->model != EMPC_PENDULUM_CHAIN)
        return fail(EMPC_EINVAL, "unknown model %d", P->model);
    if (P->n < 1 || P->m < 1) return fail(EMPC_EINVAL, "n=%d, m=%d must be >= 1", P->n, P->m);
    if (P->T < 1 || P->T > 100000) return fail(EMPC_EINVAL, "T=%d outside [1, 100000]", P->T);
    if (P->p < 1 || P->p > P->T) return fail(EMPC_EINVAL, "p=%d outside [1, T=%d]", P->p, P->T);
    if ((!P->q && !P->Q) || (!P->r && !P->R) || !P->u_min || !P->u_max)
        return fail(EMPC_EINVAL, "q (or Q), r (or R), u_min and u_max are required");
    if (P->qb && (!P->x_min || !P->x_max))
        return fail(EMPC_EINVAL, "the state box penalty (qb) needs x_min and x_max");
    if (P->sb && !P->qb)
        return fail(EMPC_EINVAL, "the step charge (sb) needs the state box (qb, x_min, x_max)");
    if (!P->q_min != !P->q_max) return fail(EMPC_EINVAL, "q_min and q_max go together");
    if (P->q_min && P->model != EMPC_PENDULUM_CHAIN)
        return fail(EMPC_EINVAL, "joint limits (q_min, q_max) belong to the pendulum chain");
    if (P->q_min && !(P->restitution >= 0.0 && P->restitution <= 1.0))
        return fail(EMPC_EINVAL, "restitution must lie in [0, 1]");
    if (!P->fric_c != !P->fric_s) return fail(EMPC_EINVAL, "fric_c and fric_s go together");
    if (P->fric_c && P->model != EMPC_PENDULUM_CHAIN)
        return fail(EMPC_EINVAL, "dry friction (fric_c, fric_s) belongs to the pendulum chain");
    const bool full = P->Q || P->R || P->Qf;
    if (full && P->model != EMPC_LINEAR)
        return fail(EMPC_EINVAL, "full weights (Q, R, Qf) belong to the linear model");
    if (P->model == EMPC_LINEAR) {
        if (!P->Ad || !P->Bd) return fail(EMPC_EINVAL, "linear model needs Ad and Bd");
        if (P->n > Limits::MAX_N_LINEAR || P->m > Limits::MAX_M_LINEAR)
            return fail(EMPC_EUNSUPPORTED, "linear n=%d, m=%d above %d, %d", P->n, P->m,
                        Limits::MAX_N_LINEAR, Limits::MAX_M_LINEAR);
        if (full && (P->n > VALU_FULL_NMAX || P->m > VALU_FULL_MMAX))
            return fail(EMPC_EUNSUPPORTED, "full weights take n <= %d, m <= %d (n=%d, m=%d)",
                        VALU_FULL_NMAX, VALU_FULL_MMAX, P->n, P->m);
    } else {
        if (P->n != 2 * P->m) return fail(EMPC_EINVAL, "chain needs n = 2m (n=%d, m=%d)", P->n, P->m);
        if (!P->stiffness || !P->damping || !P->mass || !P->length)
            return fail(EMPC_EINVAL, "chain needs stiffness, damping, mass and length");
        if (!(P->dt > 0.0) || !isfinite(P->dt) || !isfinite(P->gravity))
            return fail(EMPC_EINVAL, "chain needs a finite dt > 0 and finite gravity");
        if (P->m > Limits::MAX_D_CHAIN)
            return fail(EMPC_EUNSUPPORTED, "chain d=%d above %d", P->m, Limits::MAX_D_CHAIN);
    }
    return EMPC_OK;
}

empc_status validate_grad(const empc_problem *P) {
    if (P->Q || P->R || P->Qf)
        return fail(EMPC_EUNSUPPORTED, "the adjoint takes diagonal weights (no Q, R, Qf)");
    if (P->q_min)
        return fail(EMPC_EUNSUPPORTED, "the adjoint has no derivative through impacts (q_min, q_max)");
    if (P->fric_c)
        return fail(EMPC_EUNSUPPORTED, "the adjoint has no derivative through dry friction");
    if (P->model == EMPC_LINEAR ? P->n > 64 : P->m > 64)
        return fail(EMPC_EUNSUPPORTED, "adjoint supports n <= 64 (linear) or d <= 64 (chain)");
    const size_t b = grad_smem_bytes(P->model, P->n, P->m, P->T, P->p, esize(P));
    if (b > MAX_GRAD_LDS)
        return fail(EMPC_EUNSUPPORTED, "adjoint needs %zu bytes of LDS, above %zu", b, MAX_GRAD_LDS);
    return EMPC_OK;
}

empc_status validate_ga(const empc_ga *G) {
    if (!G) return fail(EMPC_EINVAL, "ga is NULL");
    if (G->pop < 1 || G->pop > (1 << 24)) return fail(EMPC_EINVAL, "pop=%d outside [1, 2^24]", G->pop);
    if (G->n_elite < 1 || G->n_elite > G->pop)
        return fail(EMPC_EINVAL, "n_elite=%d outside [1, pop=%d]", G->n_elite, G->pop);
    if (G->n_elite > Limits::MAX_ELITE)
        return fail(EMPC_EUNSUPPORTED, "n_elite=%d above %d", G->n_elite, Limits::MAX_ELITE);
    if (G->generations < 1) return fail(EMPC_EINVAL, "generations=%d must be >= 1", G->generations);
    if (!(G->sigma >= 0.0) || !isfinite(G->sigma)) return fail(EMPC_EINVAL, "sigma must be finite, >= 0");
    if (G->shift != 0 && G->shift != 1) return fail(EMPC_EINVAL, "shift=%d must be 0 or 1", G->shift);
    if (!(G->sigma_min >= 0.0) || !isfinite(G->sigma_min))
        return fail(EMPC_EINVAL, "sigma_min must be finite, >= 0");
    if (!(G->sigma_dist >= 0.0) || !isfinite(G->sigma_dist))
        return fail(EMPC_EINVAL, "sigma_dist must be finite, >= 0");
    return EMPC_OK;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Workspace of empc_solve, in order: header (has_elites, best_slot), two
// population buffers [pm][pop] (generation g writes buffer g % 2 and reads
// its parents in place from the other one), costs [pop], elite knots [pm][k]
// (the parents carried to the next tick), elite costs [k], elite indices
// [k] (int64), best index (int64), and the parents as a structure of arrays
// [pm][k] for gradient refinement; for a linear problem without the state
// box whose quadratic form (Sec. IV-B) fits in QP_REFINE_MAX_BYTES, that
// form too: P [pm][pm], q [pm], c, and the unit-knot responses it is built
// from (refinement then runs on the form instead of the adjoint).
struct Workspace {
    int *has_elites, *best_slot;
    void *knots[2], *cost, *elite_rows, *elite_cost, *elite_soa;
    int64_t *elite_idx, *best_idx;
    void *qP = nullptr, *qq = nullptr, *qc = nullptr, *qws = nullptr;  // quadratic form
    size_t bytes;
};

constexpr size_t QP_REFINE_MAX_BYTES = 48ull << 20;

// the linear-quadratic case whose parents refine on the quadratic form
bool quadratic_refine(const empc_problem *P) {
    if (P->model != EMPC_LINEAR || P->qb || P->Q || P->R || P->Qf) return false;
    const int pm = P->p * P->m;
    if (pm > QP_REFINE_MAX_PM) return false;
    return qp_form_bytes(P->n, P->T, pm) + (size_t)pm * pm * esize(P) <= QP_REFINE_MAX_BYTES;
}

// qp: room for the quadratic form of refinement (the static solve, which
// never refines, leaves it out)
Workspace layout(const empc_problem *P, const empc_ga *G, void *base, bool qp = true) {
    const size_t es = esize(P), pm = (size_t)P->p * P->m, pop = G->pop, k = G->n_elite;
    char *b = (char *)base;
    size_t off = 0;
    Workspace w;
    w.has_elites = (int *)(b + off);
    w.best_slot = (int *)(b + off + sizeof(int));
    off += 256;
    w.knots[0] = b + off; off += align256(pm * pop * es);
    w.knots[1] = b + off; off += align256(pm * pop * es);
    w.cost = b + off; off += align256(pop * es);
    w.elite_rows = b + off; off += align256(k * pm * es);
    w.elite_cost = b + off; off += align256(k * es);
    w.elite_idx = (int64_t *)(b + off); off += align256(k * sizeof(int64_t));
    w.best_idx = (int64_t *)(b + off); off += 256;
    w.elite_soa = b + off; off += align256(k * pm * es);
    if (qp && quadratic_refine(P)) {
        w.qP = b + off; off += align256(pm * pm * es);
        w.qq = b + off; off += align256(pm * es);
        w.qc = b + off; off += 256;
        w.qws = b + off; off += align256(qp_form_bytes(P->n, P->T, (int)pm));
    }
    w.bytes = off;
    return w;
}

// Rollout timing with HIP events (empc_profile_begin / _end).
struct Profile {
    bool on = false;
    int used = 0;
    std::vector<hipEvent_t> start, stop;
};
Profile g_prof;

// Timing events for the next rollout launch of an open profiling session.
Events next_events() {
    Events ev;
    if (g_prof.on && g_prof.used < (int)g_prof.start.size()) {
        ev.start = g_prof.start[g_prof.used];
        ev.stop = g_prof.stop[g_prof.used];
        ++g_prof.used;
    }
    return ev;
}

// Tuning table of the single-problem path (empc_autotune): per problem
// shape and candidate count, the rollout form and the population's
// parameter groups per workgroup.  Shapes not in the table use the fixed
// rules.  Every lookup and update holds the mutex.
typedef std::tuple<int, int, int, int, int, int, int64_t, int, int, int, int> TuneKey;
struct Tuned {
    int form = RF_RULE;
    int R = 0;
};
std::mutex g_tune_mu;
std::map<TuneKey, Tuned> g_tune;

TuneKey tune_key(const empc_problem *P, int64_t ncand) {
    return TuneKey(P->model, P->dtype, P->n, P->m, P->T, P->p, ncand, P->qb ? 1 : 0,
                   P->x_goal ? 1 : 0, P->wd ? 1 : 0,
                   ((P->Q || P->R || P->Qf) ? 1 : 0) | (P->q_min ? 2 : 0) |
                       (P->fric_c ? 4 : 0));
}
Tuned tuned_for(const empc_problem *P, int64_t ncand) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_tune.find(tune_key(P, ncand));
    return it == g_tune.end() ? Tuned() : it->second;
}

template <typename T>
hipError_t timed_rollout(const ProbView<T> &V, int model, const T *x0, const T *knots,
                         int64_t ncand, int64_t ld, T *cost, hipStream_t s, int form = RF_RULE) {
    return launch_rollout<T>(V, model, x0, knots, ncand, ld, cost, s, next_events(), form);
}

// Gradient refinement of the parents after a selection: Adam on the
// parents, which land in elite_soa ([pm][k], the layout of the parent rows:
// the next generation's population reads them there); after the last
// generation the parent rows for the next tick, u* and the best cost.
template <typename T>
hipError_t refine_parents(const empc_problem *P, const empc_ga *G, const Workspace &w,
                          const void *x0, const T *cur, double lr, int steps, bool last,
                          void *u_star, void *best_cost, hipStream_t s) {
    const ProbView<T> V = view_of<T>(*P);
    const int k = G->n_elite, pm = P->p * P->m;
    hipError_t e;
    if (w.qP) {  // on the quadratic form of this tick (built before generation 0)
        e = launch_qp_refine<T>(V, (const T *)w.qP, (const T *)w.qq, (const T *)w.qc, cur,
                                G->pop, w.elite_idx, (T *)w.elite_soa, k, steps, (T)lr,
                                (T *)w.elite_cost, s);
    } else {
        e = launch_gather_parents<T>(cur, G->pop, w.elite_idx, k, pm, (T *)w.elite_soa, s);
        if (e == hipSuccess)
            e = launch_grad<T>(V, P->model, (const T *)x0, nullptr, k, k, nullptr, nullptr,
                               steps, (T)lr, (T *)w.elite_soa, (T *)w.elite_cost, s);
    }
    if (e != hipSuccess || !last) return e;
    return launch_finish_refine<T>((const T *)w.elite_soa, k, pm, P->m, (const T *)w.elite_cost,
                                   (T *)w.elite_rows, w.best_slot, last ? (T *)u_star : nullptr,
                                   last ? (T *)best_cost : nullptr, s);
}

template <typename T>
empc_status solve_t(const empc_problem *P, const empc_ga *G, const Workspace &w, const void *x0,
                    uint32_t tick, void *u_star, void *best_cost, hipStream_t s,
                    int adam_steps = 0, double lr = 0.0) {
    const ProbView<T> V = view_of<T>(*P);
    const int64_t pop = G->pop;
    const bool refine = adam_steps > 0;
    const Tuned tu = tuned_for(P, pop);
    if (refine && w.qP) {  // the quadratic form at this tick's x0 (the model may change per tick)
        const hipError_t e = launch_qp_form<T>(V, (const T *)x0, w.qws, (T *)w.qP, (T *)w.qq,
                                               (T *)w.qc, s);
        if (e != hipSuccess) return device_status(e, "quadratic form launch");
    }
    for (int g = 0; g < G->generations; ++g) {
        const bool last = g == G->generations - 1;
        T *cur = (T *)w.knots[g & 1];
        const T *prev = (const T *)w.knots[(g + 1) & 1];
        // generation 0 starts from the parents carried over from the last
        // tick (or cold-starts); later ones read their parents in place
        // (with refinement the parents are always the refined parent rows)
        // (the optional shift moves the carried parents once, at generation 0)
        const PopVariant<T> var = pop_variant<T>(*G, x0, g == 0);
        // (refined parents of the previous generation: elite_soa, same layout)
        const T *rows = (g > 0 && refine) ? (const T *)w.elite_soa : (const T *)w.elite_rows;
        hipError_t e = (g == 0 || refine)
                           ? launch_population<T>(V, *G, nullptr, 0, nullptr, rows, w.has_elites,
                                                  g == 0 ? 2 : 0, cur, pop, tick, (uint32_t)g, s,
                                                  var, tu.R)
                           : launch_population<T>(V, *G, prev, pop, w.elite_idx, nullptr,
                                                  nullptr, 0, cur, pop, tick, (uint32_t)g, s, var,
                                                  tu.R);
        if (e != hipSuccess) return device_status(e, "population launch");
        e = timed_rollout<T>(V, P->model, (const T *)x0, cur, pop, pop, (T *)w.cost, s, tu.form);
        if (e != hipSuccess) return device_status(e, "rollout launch");
        e = launch_select<T>(V, (const T *)w.cost, cur, pop, pop, G->n_elite, w.elite_idx,
                             w.best_idx, (last && !refine) ? (T *)w.elite_rows : nullptr,
                             (T *)w.elite_cost, w.has_elites, w.best_slot,
                             (last && !refine) ? (T *)u_star : nullptr,
                             (last && !refine) ? (T *)best_cost : nullptr, s);
        if (e != hipSuccess) return device_status(e, "select launch");
        if (refine) {
            e = refine_parents<T>(P, G, w, x0, cur, lr, adam_steps, last, u_star, best_cost, s);
            if (e != hipSuccess) return device_status(e, "refine launch");
        }
    }
    return EMPC_OK;
}

// Mean launch time (us) of `enqueue` over reps launches after one untimed.
template <typename F>
hipError_t time_us(F &&enqueue, int reps, hipStream_t s, hipEvent_t t0, hipEvent_t t1, float *us) {
    hipError_t e = enqueue();
    if (e == hipSuccess) e = hipEventRecord(t0, s);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = enqueue();
    if (e == hipSuccess) e = hipEventRecord(t1, s);
    if (e == hipSuccess) e = hipEventSynchronize(t1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
    *us = ms * 1e3f / (float)reps;
    return e;
}

// The single-problem autotuner: time every rollout form of the shape on a
// cold-start population, then the population kernel's parameter groups per
// workgroup, and record the fastest in the tuning table.
template <typename T>
empc_status autotune_t(const empc_problem *P, const empc_ga *G, int reps, int allow_valu,
                       float *info, hipStream_t s) {
    const ProbView<T> V = view_of<T>(*P);
    const int64_t pop = G->pop;
    const int pm = P->p * P->m, k = G->n_elite;
    T *knots = nullptr, *knots2 = nullptr, *cost = nullptr, *x0 = nullptr;
    int64_t *eidx = nullptr;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    hipError_t e = hipMalloc(&knots, sizeof(T) * pm * pop);
    if (e == hipSuccess) e = hipMalloc(&knots2, sizeof(T) * pm * pop);
    if (e == hipSuccess) e = hipMalloc(&cost, sizeof(T) * pop);
    if (e == hipSuccess) e = hipMalloc(&x0, sizeof(T) * P->n);
    if (e == hipSuccess) e = hipMalloc(&eidx, sizeof(int64_t) * k);
    if (e == hipSuccess) e = hipEventCreate(&t0);
    if (e == hipSuccess) e = hipEventCreate(&t1);
    if (e == hipSuccess) e = hipMemsetAsync(x0, 0, sizeof(T) * P->n, s);
    if (e == hipSuccess) {
        std::vector<int64_t> idx(k);
        for (int i = 0; i < k; ++i) idx[i] = (int64_t)i * (pop / k);
        e = hipMemcpyAsync(eidx, idx.data(), sizeof(int64_t) * k, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    if (e == hipSuccess)
        e = launch_population<T>(V, *G, nullptr, 0, nullptr, nullptr, nullptr, 1, knots, pop, 0, 0, s);
    std::vector<int> forms;
    if (P->model == EMPC_LINEAR && (P->Q || P->R || P->Qf)) {
        // full weights: the 16-lane row form (the rule) or, small, the VALU form
        if (P->n <= 16 && P->m <= 16) forms = {RF_VALU256, RF_VALU64};
    } else if (P->model == EMPC_LINEAR) {
        forms = {RF_ONE1, RF_ONE2, RF_ONE4};
        if (P->n > 16) forms.push_back(RF_SPLIT);
        if (allow_valu && P->n <= 16 && P->m <= 16) {
            forms.push_back(RF_VALU256);
            forms.push_back(RF_VALU64);
        }
    } else {
        forms = {RF_CH64, RF_CH128, RF_CH256};
    }
    float rule_us = 0.f, best_us = 0.f;
    int best_form = RF_RULE;
    auto rollout = [&](int form) {
        return launch_rollout<T>(V, P->model, x0, knots, pop, pop, cost, s, Events(), form);
    };
    if (e == hipSuccess) e = time_us([&]() { return rollout(RF_RULE); }, reps, s, t0, t1, &rule_us);
    best_us = rule_us;
    for (int f : forms) {
        if (e != hipSuccess) break;
        float us = 0.f;
        e = time_us([&]() { return rollout(f); }, reps, s, t0, t1, &us);
        if (e == hipSuccess && us < best_us) {
            best_us = us;
            best_form = f;
        }
    }
    // population: parameter groups per workgroup (the same bits for each)
    float pop_best = 0.f;
    int best_R = 0;
    for (int R : {1, 2, 4}) {
        if (e != hipSuccess) break;
        float us = 0.f;
        e = time_us([&]() {
                return launch_population<T>(V, *G, knots, pop, eidx, nullptr, nullptr, 0, knots2,
                                            pop, 1, 1, s, PopVariant<T>(), R);
            }, reps, s, t0, t1, &us);
        if (e == hipSuccess && (best_R == 0 || us < pop_best)) {
            pop_best = us;
            best_R = R;
        }
    }
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    (void)hipFree(knots);
    (void)hipFree(knots2);
    (void)hipFree(cost);
    (void)hipFree(x0);
    (void)hipFree(eidx);
    if (e != hipSuccess) return device_status(e, "autotune");
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        Tuned t;
        t.form = best_form;
        t.R = best_R;
        g_tune[tune_key(P, pop)] = t;
    }
    if (info) {
        info[0] = (float)best_form;
        info[1] = (float)best_R;
        info[2] = best_us;
        info[3] = rule_us;
        info[4] = pop_best;
    }
    return EMPC_OK;
}

// Workspace of empc_solve_static: one array per GPU, held from the load of
// the library's code object to the end of the process.  In host code the
// symbol is only a host-side stand-in; its device address is looked up once
// per device (with that device current) and used everywhere instead.
__device__ __align__(256) unsigned char scratch[EMPC_STATIC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[MAX_DEVICES] = {};

empc_status static_scratch(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return device_status(e, "hipGetDevice");
    if (dev < 0 || dev >= MAX_DEVICES) return fail(EMPC_EUNSUPPORTED, "device %d above %d", dev, MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return device_status(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(EMPC_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return EMPC_OK;
}

// Clears the warm-start words of a solve workspace header (a kernel, not a
// memset, so that a captured graph replays it as it was recorded).
__global__ void clear_header_kernel(int *head) {
    if (threadIdx.x < 2) head[threadIdx.x] = 0;
}

}  // namespace

empc_status empc_validate_problem_internal(const empc_problem *P) { return validate_problem(P); }
empc_status empc_validate_ga_internal(const empc_ga *G) { return validate_ga(G); }
empc_status empc_fail_internal(empc_status s, const char *msg) { return fail(s, "%s", msg); }

extern "C" {

const char *empc_status_str(empc_status s) {
    switch (s) {
        case EMPC_OK: return "ok";
        case EMPC_EINVAL: return "invalid argument";
        case EMPC_EDEVICE: return "device error";
        case EMPC_EUNSUPPORTED: return "unsupported problem size";
        case EMPC_EWORKSPACE: return "workspace too small";
    }
    return "unknown status";
}

const char *empc_last_error(void) { return g_err; }

empc_status empc_rollout_cost(const empc_problem *prob, const void *x0, const void *knots,
                              int64_t ncand, int64_t ld, void *cost, void *stream) {
    empc_status st = validate_problem(prob);
    if (st) return st;
    if (ncand < 0 || ld < ncand) return fail(EMPC_EINVAL, "need 0 <= ncand <= ld (ncand=%lld, ld=%lld)",
                                             (long long)ncand, (long long)ld);
    if (ncand == 0) return EMPC_OK;
    if (!x0 || !knots || !cost) return fail(EMPC_EINVAL, "x0, knots and cost are required");
    if ((st = check_prior())) return st;
    hipStream_t s = (hipStream_t)stream;
    const int form = tuned_for(prob, ncand).form;
    hipError_t e = prob->dtype == EMPC_F32
                       ? timed_rollout<float>(view_of<float>(*prob), prob->model, (const float *)x0,
                                              (const float *)knots, ncand, ld, (float *)cost, s,
                                              form)
                       : timed_rollout<double>(view_of<double>(*prob), prob->model,
                                                (const double *)x0, (const double *)knots, ncand, ld,
                                                (double *)cost, s, form);
    return device_status(e, "rollout launch");
}

empc_status empc_generation(const empc_problem *prob, const empc_ga *ga, const void *knots_in,
                            int64_t ld_in, const void *cost_in, void *knots_out, int64_t ld_out,
                            int64_t *elite_idx, int64_t *best_idx, uint32_t tick, uint32_t gen,
                            void *stream) {
    empc_status st = validate_problem(prob);
    if (st) return st;
    if ((st = validate_ga(ga))) return st;
    const bool cold = knots_in == nullptr && cost_in == nullptr;
    if (!knots_out) return fail(EMPC_EINVAL, "knots_out is required");
    if (ld_out < ga->pop) return fail(EMPC_EINVAL, "ld_out=%lld < pop=%d", (long long)ld_out, ga->pop);
    if (!cold) {
        if (!knots_in || !cost_in) return fail(EMPC_EINVAL, "knots_in and cost_in go together");
        if (!elite_idx) return fail(EMPC_EINVAL, "elite_idx is required for a warm start");
        if (ld_in < ga->pop) return fail(EMPC_EINVAL, "ld_in=%lld < pop=%d", (long long)ld_in, ga->pop);
        const size_t es = esize(prob), pm = (size_t)prob->p * prob->m;
        const char *a0 = (const char *)knots_in, *a1 = a0 + ((pm - 1) * ld_in + ga->pop) * es;
        const char *b0 = (const char *)knots_out, *b1 = b0 + ((pm - 1) * ld_out + ga->pop) * es;
        if (a0 < b1 && b0 < a1) return fail(EMPC_EINVAL, "knots_out overlaps knots_in");
    }
    if ((st = check_prior())) return st;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    if (prob->dtype == EMPC_F32) {
        const ProbView<float> V = view_of<float>(*prob);
        if (!cold) {
            e = launch_select<float>(V, (const float *)cost_in, (const float *)knots_in, ld_in,
                                     ga->pop, ga->n_elite, elite_idx, best_idx, nullptr, nullptr,
                                     nullptr, nullptr, nullptr, nullptr, s);
            if (e != hipSuccess) return device_status(e, "select launch");
        }
        e = launch_population<float>(V, *ga, (const float *)knots_in, ld_in, elite_idx, nullptr,
                                     nullptr, cold ? 1 : 0, (float *)knots_out, ld_out, tick, gen, s);
    } else {
        const ProbView<double> V = view_of<double>(*prob);
        if (!cold) {
            e = launch_select<double>(V, (const double *)cost_in, (const double *)knots_in, ld_in,
                                      ga->pop, ga->n_elite, elite_idx, best_idx, nullptr, nullptr,
                                      nullptr, nullptr, nullptr, nullptr, s);
            if (e != hipSuccess) return device_status(e, "select launch");
        }
        e = launch_population<double>(V, *ga, (const double *)knots_in, ld_in, elite_idx, nullptr,
                                      nullptr, cold ? 1 : 0, (double *)knots_out, ld_out, tick, gen,
                                      s);
    }
    return device_status(e, "population launch");
}

size_t empc_workspace_bytes(const empc_problem *prob, const empc_ga *ga) {
    if (validate_problem(prob) || validate_ga(ga)) return 0;
    return layout(prob, ga, nullptr).bytes;
}

empc_status empc_solve(const empc_problem *prob, const empc_ga *ga, void *workspace,
                       size_t ws_bytes, const void *x0, uint32_t tick, void *u_star,
                       void *best_cost, void *stream) {
    empc_status st = validate_problem(prob);
    if (st) return st;
    if ((st = validate_ga(ga))) return st;
    if (!x0 || !u_star || !best_cost) return fail(EMPC_EINVAL, "x0, u_star and best_cost are required");
    const Workspace w = layout(prob, ga, workspace);
    if (!workspace || ws_bytes < w.bytes)
        return fail(EMPC_EWORKSPACE, "workspace of %zu bytes, need %zu", ws_bytes, w.bytes);
    if ((st = check_prior())) return st;
    hipStream_t s = (hipStream_t)stream;
    return prob->dtype == EMPC_F32 ? solve_t<float>(prob, ga, w, x0, tick, u_star, best_cost, s)
                                   : solve_t<double>(prob, ga, w, x0, tick, u_star, best_cost, s);
}

empc_status empc_solve_refined(const empc_problem *prob, const empc_ga *ga, void *workspace,
                               size_t ws_bytes, const void *x0, uint32_t tick, double lr,
                               int32_t adam_steps, void *u_star, void *best_cost, void *stream) {
    empc_status st = validate_problem(prob);
    if (st) return st;
    if ((st = validate_ga(ga))) return st;
    if (adam_steps < 1 || !(lr >= 0.0) || !isfinite(lr))
        return fail(EMPC_EINVAL, "need adam_steps >= 1 and a finite lr >= 0");
    // (the parents of a linear-quadratic problem refine on its quadratic
    // form, whatever its size; the others need the adjoint's limits)
    if (!quadratic_refine(prob) && (st = validate_grad(prob))) return st;
    if (!x0 || !u_star || !best_cost) return fail(EMPC_EINVAL, "x0, u_star and best_cost are required");
    const Workspace w = layout(prob, ga, workspace);
    if (!workspace || ws_bytes < w.bytes)
        return fail(EMPC_EWORKSPACE, "workspace of %zu bytes, need %zu", ws_bytes, w.bytes);
    if ((st = check_prior())) return st;
    hipStream_t s = (hipStream_t)stream;
    return prob->dtype == EMPC_F32
               ? solve_t<float>(prob, ga, w, x0, tick, u_star, best_cost, s, adam_steps, lr)
               : solve_t<double>(prob, ga, w, x0, tick, u_star, best_cost, s, adam_steps, lr);
}

empc_status empc_solve_static(const empc_problem *prob, const empc_ga *ga, const void *x0,
                              uint32_t tick, int32_t cold, void *u_star, void *best_cost,
                              void *stream) {
    empc_status st = validate_problem(prob);
    if (st) return st;
    if ((st = validate_ga(ga))) return st;
    if (cold != 0 && cold != 1) return fail(EMPC_EINVAL, "cold=%d must be 0 or 1", cold);
    if (!x0 || !u_star || !best_cost) return fail(EMPC_EINVAL, "x0, u_star and best_cost are required");
    const size_t need = layout(prob, ga, nullptr, false).bytes;
    if (need > EMPC_STATIC_SCRATCH_BYTES)
        return fail(EMPC_EUNSUPPORTED, "solve needs %zu bytes of workspace, above the static %zu",
                    need, (size_t)EMPC_STATIC_SCRATCH_BYTES);
    if ((st = check_prior())) return st;
    void *base = nullptr;
    if ((st = static_scratch(&base))) return st;
    hipStream_t s = (hipStream_t)stream;
    const Workspace w = layout(prob, ga, base, false);
    if (cold) {
        hipLaunchKernelGGL(clear_header_kernel, dim3(1), dim3(64), 0, s, w.has_elites);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return device_status(e, "clear launch");
    }
    return prob->dtype == EMPC_F32 ? solve_t<float>(prob, ga, w, x0, tick, u_star, best_cost, s)
                                   : solve_t<double>(prob, ga, w, x0, tick, u_star, best_cost, s);
}

empc_status empc_autotune(const empc_problem *prob, const empc_ga *ga, int32_t reps,
                          int32_t allow_valu, float *info, void *stream) {
    empc_status st = validate_problem(prob);
    if (st) return st;
    if ((st = validate_ga(ga))) return st;
    if (reps < 1) return fail(EMPC_EINVAL, "reps must be >= 1");
    if ((st = check_prior())) return st;
    hipStream_t s = (hipStream_t)stream;
    return prob->dtype == EMPC_F32 ? autotune_t<float>(prob, ga, reps, allow_valu, info, s)
                                   : autotune_t<double>(prob, ga, reps, allow_valu, info, s);
}

empc_status empc_autotune_set(const empc_problem *prob, const empc_ga *ga, int32_t form,
                              int32_t groups) {
    empc_status st = validate_problem(prob);
    if (st) return st;
    if ((st = validate_ga(ga))) return st;
    const bool lin = prob->model == EMPC_LINEAR;
    const bool ok = form == RF_RULE ||
                    (lin && (form == RF_ONE1 || form == RF_ONE2 || form == RF_ONE4 ||
                             form == RF_SPLIT || form == RF_VALU256 || form == RF_VALU64)) ||
                    (!lin && (form == RF_CH64 || form == RF_CH128 || form == RF_CH256));
    if (!ok) return fail(EMPC_EINVAL, "rollout form %d does not exist for this model", form);
    if (groups != 0 && groups != 1 && groups != 2 && groups != 4)
        return fail(EMPC_EINVAL, "groups=%d must be 0, 1, 2 or 4", groups);
    const bool full = prob->Q || prob->R || prob->Qf;
    if ((form == RF_VALU256 || form == RF_VALU64) && (prob->n > 16 || prob->m > 16))
        return fail(EMPC_EUNSUPPORTED, "the vector-ALU form takes n, m <= 16");
    if (full && form != RF_RULE && form != RF_VALU256 && form != RF_VALU64)
        return fail(EMPC_EUNSUPPORTED,
                     "full weights run the 16-lane row form (the rule) or the vector-ALU form");
    if (form == RF_SPLIT && prob->n <= 16)
        return fail(EMPC_EUNSUPPORTED, "the M-split form needs more than 16 states");
    std::lock_guard<std::mutex> lock(g_tune_mu);
    Tuned t;
    t.form = form;
    t.R = groups;
    g_tune[tune_key(prob, ga->pop)] = t;
    return EMPC_OK;
}

empc_status empc_autotune_reset(void) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune.clear();
    return EMPC_OK;
}

empc_status empc_grad(const empc_problem *prob, const void *x0, const void *knots, int64_t ncand,
                      int64_t ld, void *dJ, void *cost, void *stream) {
    empc_status st = validate_problem(prob);
    if (st) return st;
    if (ncand < 0 || ld < ncand) return fail(EMPC_EINVAL, "need 0 <= ncand <= ld");
    if (ncand == 0) return EMPC_OK;
    if (!x0 || !knots || !dJ) return fail(EMPC_EINVAL, "x0, knots and dJ are required");
    if ((st = validate_grad(prob))) return st;
    if ((st = check_prior())) return st;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = prob->dtype == EMPC_F32
                       ? launch_grad<float>(view_of<float>(*prob), prob->model, (const float *)x0,
                                            (const float *)knots, ncand, ld, (float *)dJ,
                                            (float *)cost, 0, 0.f, nullptr, nullptr, s)
                       : launch_grad<double>(view_of<double>(*prob), prob->model,
                                             (const double *)x0, (const double *)knots, ncand, ld,
                                             (double *)dJ, (double *)cost, 0, 0.0, nullptr, nullptr,
                                             s);
    return device_status(e, "grad launch");
}

empc_status empc_refine(const empc_problem *prob, const void *x0, void *knots, int64_t ncand,
                        int64_t ld, void *cost, double lr, int32_t steps, void *stream) {
    empc_status st = validate_problem(prob);
    if (st) return st;
    if (ncand < 0 || ld < ncand) return fail(EMPC_EINVAL, "need 0 <= ncand <= ld");
    if (steps < 0 || !(lr >= 0.0) || !isfinite(lr)) return fail(EMPC_EINVAL, "need steps >= 0, finite lr >= 0");
    if (ncand == 0 || steps == 0) return EMPC_OK;
    if (!x0 || !knots || !cost) return fail(EMPC_EINVAL, "x0, knots and cost are required");
    if ((st = validate_grad(prob))) return st;
    if ((st = check_prior())) return st;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = prob->dtype == EMPC_F32
                       ? launch_grad<float>(view_of<float>(*prob), prob->model, (const float *)x0,
                                            nullptr, ncand, ld, nullptr, nullptr, steps, (float)lr,
                                            (float *)knots, (float *)cost, s)
                       : launch_grad<double>(view_of<double>(*prob), prob->model,
                                             (const double *)x0, nullptr, ncand, ld, nullptr,
                                             nullptr, steps, lr, (double *)knots, (double *)cost, s);
    return device_status(e, "refine launch");
}

empc_status empc_plant_step(const empc_problem *prob, const void *x, const void *u,
                            const void *noise, void *x_next, void *stream) {
    empc_status st = validate_problem(prob);
    if (st) return st;
    if (!x || !u || !x_next) return fail(EMPC_EINVAL, "x, u and x_next are required");
    if ((st = check_prior())) return st;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = prob->dtype == EMPC_F32
                       ? launch_plant<float>(view_of<float>(*prob), prob->model, (const float *)x,
                                             (const float *)u, (const float *)noise,
                                             (float *)x_next, s)
                       : launch_plant<double>(view_of<double>(*prob), prob->model,
                                              (const double *)x, (const double *)u,
                                              (const double *)noise, (double *)x_next, s);
    return device_status(e, "plant launch");
}

empc_status empc_profile_begin(int32_t max_launches) {
    if (max_launches < 1) return fail(EMPC_EINVAL, "max_launches must be >= 1");
    if (g_prof.on) return fail(EMPC_EINVAL, "a profiling session is already open");
    while ((int)g_prof.start.size() < max_launches) {
        hipEvent_t a, b;
        hipError_t e = hipEventCreate(&a);
        if (e != hipSuccess) return device_status(e, "hipEventCreate");
        e = hipEventCreate(&b);
        if (e != hipSuccess) {
            (void)hipEventDestroy(a);
            return device_status(e, "hipEventCreate");
        }
        g_prof.start.push_back(a);
        g_prof.stop.push_back(b);
    }
    g_prof.used = 0;
    g_prof.on = true;
    return EMPC_OK;
}

empc_status empc_profile_end(int64_t *launches, double *total_ms) {
    if (!g_prof.on) return fail(EMPC_EINVAL, "no profiling session is open");
    g_prof.on = false;
    double tot = 0.0;
    for (int i = 0; i < g_prof.used; ++i) {
        hipError_t e = hipEventSynchronize(g_prof.stop[i]);
        if (e != hipSuccess) return device_status(e, "hipEventSynchronize");
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, g_prof.start[i], g_prof.stop[i]);
        if (e != hipSuccess) return device_status(e, "hipEventElapsedTime");
        tot += ms;
    }
    if (launches) *launches = g_prof.used;
    if (total_ms) *total_ms = tot;
    return EMPC_OK;
}

}  // extern "C"
