// nbody.hip -- libnbody: the C ABI declared in include/nbody.h, for gfx950.
//
// The host side owns only the context, its device work buffers (j-particle stream, block list,
// scheduler record, force partial sums, energy scratch) and captured HIP graphs.  All particle
// state is the caller's.  Every kernel sizes its work from device-resident counts, so a block
// step needs no host round trip and can be captured and replayed as a graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/nbody.h"
#include "adjoint.hpp"
#include "ensemble.hpp"
#include "kernels.hpp"

using namespace nbody;

// ------------------------------------------------------------------------------------------
// The j-split partial sums of nb_force_noalloc: one static device array per GPU (it lives as
// long as the process), so that call never needs device memory from the caller or the
// allocator.  Host code reaches it only through the address hipGetSymbolAddress returns for
// the device (the array's name is a host-side stand-in there).
// ------------------------------------------------------------------------------------------
namespace {
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;
static __device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];
std::mutex noalloc_mu;
void *noalloc_ptr[NOALLOC_MAX_DEVICES] = {};
bool noalloc_done[NOALLOC_MAX_DEVICES] = {};

// Once per device, with that device current: the device address of its scratch array.
void noalloc_setup(int device) {
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return;
    std::lock_guard<std::mutex> lock(noalloc_mu);
    if (noalloc_done[device]) return;
    noalloc_done[device] = true;
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess) noalloc_ptr[device] = p;
}

void *noalloc_scratch(int device) {
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(noalloc_mu);
    return noalloc_ptr[device];
}
}  // namespace

namespace {

using Variant = nb_variant;

// Compiled force-kernel variants: i-particles per work-item x j-loop unroll.
bool variant_compiled(int prec, const Variant &v) {
    const bool unr_ok = v.unroll == 1 || v.unroll == 2 || v.unroll == 4;
    if (prec == NB_FP32)
        return unr_ok && (v.ipl == 1 || v.ipl == 2 || (v.ipl == 4 && v.unroll <= 2));
    if (prec == NB_FP32_FIXED) return (v.ipl == 1 || v.ipl == 2) && (v.unroll == 1 || v.unroll == 2);
    // NB_FP32_ALL, NB_DS, NB_FP64
    return v.ipl == 1 && (v.unroll == 1 || v.unroll == 2);
}

}  // namespace

struct nb_ctx {
    int32_t n = 0;
    double eps = 0.0;
    int32_t lmin = 0, lmax = 0, prec = 0;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;  // private stream used only to capture graphs
    nb_state st{};
    bool bound = false;
    bool predicted = false;
    bool forced = false;
    int device = 0;
    int num_cu = 256;

    // device work buffers, carved from the caller's workspace by nb_bind_scratch()
    bool scratch_ok = false;
    size_t scratch_need = 0;
    void *jbuf = nullptr;
    JStreamView js{};
    double *acc1 = nullptr, *jerk1 = nullptr, *pot1 = nullptr;  // block force outputs, ld = n
    double *partial = nullptr;
    int64_t partial_rows = 0;
    int32_t *active = nullptr;
    double *crit = nullptr;
    int64_t *wgmin = nullptr;
    int32_t *cnt = nullptr;
    DevControl *ctl = nullptr;
    double *exp_ = nullptr, *evp = nullptr, *ew = nullptr, *ek = nullptr, *eout = nullptr;
    int64_t *t_zero = nullptr;
    double *adj = nullptr;  // a1_bar, k1_bar, xp_bar, vp_bar (3n each) for the step VJP
    int32_t *adj_flag = nullptr;

    int32_t sched_groups = 1, sched_chunk = 1;
    int32_t fused_groups = 1, fused_chunk = 1;  // chunks of the fused step's count + predict
    int32_t resident_max = 1024;         // nb_run: one resident workgroup up to this n
    Variant var_full{2, 2, 4096, 256, 16};   // calls on (nearly) all particles
    Variant var_block{2, 2, 4096, 256, 16};  // block-step calls (device-resident count)
    int32_t max_target = 4096;           // partial planes are sized for targets up to this
    int32_t *tune_n = nullptr;           // device count used while tuning

    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    double graph_eta = -1.0;
    int32_t graph_steps = 0;

    // force-kernel timing (HIP events on the context stream), off by default
    bool profile = false;
    struct Timed {
        hipEvent_t start, stop;
        int cls;
    };
    std::vector<Timed> ev;

    std::string err;
};

// Most independent lanes of an ensemble: each runs on a stream of its own, and a process gets
// four hardware queues, one of which the caller's stream keeps.
constexpr int ENS_MAX_LANES = 3;

struct nb_ens {
    int32_t C = 0, ntot = 0, lmin = 0, lmax = 0, prec = 0;
    int device = 0, num_cu = 256;
    hipStream_t stream = nullptr, cap_stream = nullptr;
    nb_state st{};
    bool bound = false, initialised = false;
    std::vector<int32_t> off_h, tpi_h, K_h, prow_h, order_h;
    std::vector<int64_t> part_off_h;
    std::vector<double> eps2_h;
    int32_t *off = nullptr, *K = nullptr, *tpi = nullptr, *prow = nullptr, *active = nullptr;
    int32_t *order = nullptr;
    int32_t *flags = nullptr;
    int64_t *part_off = nullptr;
    double *eps2 = nullptr, *partial = nullptr, *crit = nullptr, *ek = nullptr, *ep = nullptr;
    EnsCluster *cl = nullptr;
    bool scratch_ok = false;
    size_t scratch_need = 0;
    int32_t unroll = 2, grid_force = 1;
    // blocks the clusters' own workgroups advance (see ens_local_block)
    int64_t local_limit = 0, local_work = 1 << 21;
    int32_t local_steps = 64;
    int32_t smin = 8;  // fewest lanes per block particle in a force item
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    double g_eta = -1.0;
    int64_t g_tend = -1;
    int32_t g_steps = 0;
    // independent lanes (nb_ens_set_lanes): lane l advances the clusters at places
    // [lane_start_h[l], lane_start_h[l + 1]) of order_h by a graph of its own on a stream of its
    // own, so its global steps follow only its clusters' block times
    int32_t lanes = 1;
    std::vector<int32_t> size_order_h, lane_start_h;
    hipStream_t lane_stream[ENS_MAX_LANES] = {};
    hipEvent_t lane_event[ENS_MAX_LANES] = {};
    hipEvent_t lane_join = nullptr;
    hipGraphExec_t lane_gexec[ENS_MAX_LANES] = {};
    hipGraph_t lane_graph[ENS_MAX_LANES] = {};
    EnsCluster *lane_host[ENS_MAX_LANES] = {};  // pinned copies of the cluster records
    std::string err;
};

namespace {

nb_status fail(nb_ens *e, nb_status s, const char *fmt, ...) {
    if (e) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        e->err = buf;
    }
    return s;
}

nb_status fail(nb_ctx *c, nb_status s, const char *fmt, ...) {
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return s;
}

#define HIP_OK(ctx, call)                                                                    \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail((ctx), NB_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));   \
    } while (0)

#define LAUNCH_OK(ctx)                                                                       \
    do {                                                                                     \
        hipError_t e_ = hipGetLastError();                                                   \
        if (e_ != hipSuccess)                                                                \
            return fail((ctx), NB_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e_)); \
    } while (0)

int32_t grid_for(int64_t n, int32_t cap) {
    int64_t g = (n + WG - 1) / WG;
    if (g < 1) g = 1;
    return (int32_t)std::min<int64_t>(g, cap);
}

StateView state_view(const nb_ctx *c) {
    return StateView{c->st.x, c->st.v, c->st.a, c->st.k, c->st.m, c->st.tick, c->n,
                     std::ldexp(1.0, -c->lmax)};
}

StateRW state_rw(const nb_ctx *c) {
    return StateRW{c->st.x, c->st.v, c->st.a, c->st.k, c->st.m, c->st.pot, c->st.tick,
                   c->st.level, c->n, std::ldexp(1.0, -c->lmax)};
}

SchedView fused_view(const nb_ctx *c) {
    return SchedView{c->st.tick, c->st.level, c->n, c->lmax, c->fused_chunk, c->fused_groups,
                     c->wgmin, c->cnt, c->active};
}

SchedView sched_view(const nb_ctx *c) {
    return SchedView{c->st.tick, c->st.level, c->n, c->lmax, c->sched_chunk, c->sched_groups,
                     c->wgmin, c->cnt, c->active};
}

// Work-item targets: up to FULL_ITEMS_PER_CU per compute unit with at most FULL_KMAX j-ranges
// (the full-force class), or up to BLOCK_ITEMS_PER_CU with any split; partial planes are sized
// for both families.
constexpr int32_t FULL_ITEMS_PER_CU = 256, FULL_KMAX = 64, BLOCK_ITEMS_PER_CU = 16;

// Heuristic defaults per size class; nb_tune() replaces them with measured choices.
Variant default_variant(int32_t n, int prec, int num_cu, bool block) {
    Variant v;
    // measured on MI355X: full-force calls at N = 2^20 take one i per work-item, unroll 2 and
    // 256 work items per compute unit (FP32 with scalar j-loads: 601-605 ms, against 612 ms at
    // 128 per CU and 622 ms at 64; K = 16 j-ranges of 2.6 MB, so that the XCD streaming one
    // range holds it in its 4 MB L2; two i per work-item and unroll 1: 616 ms at 128 per CU),
    // with the j-split capped at 64 ranges; block
    // steps (N = 65536 run, every block size from 1 to N) take one i per work-item, unroll 2
    // and 16 items per compute unit (more, shorter items at every block size)
    v.ipl = 1;
    v.unroll = 2;
    v.target = num_cu * (block ? BLOCK_ITEMS_PER_CU : FULL_ITEMS_PER_CU);
    v.kmax = block ? 1 << 16 : FULL_KMAX;  // K is also bounded by the tile count
    // scalar j-loads from 1 tile per item in full-force calls and from 4 in block steps
    // (interleaved runs on one MI355X against 16 tiles: the shared-step gradient at N = 16384,
    // whose full forces are one-tile items, 54.3 against 56.1 ms; the N = 65536 block-step run
    // 2.73 against 2.79 s, where 1 tile gave 2.80 s and 8 tiles 2.75 s)
    v.scalar_tiles = block ? 4 : 1;
    if (block || (prec != NB_FP32 && prec != NB_FP32_FIXED)) return v;
    // full-force calls of 2^16 and 2^17 particles (force + reduction per call, warm clocks, the
    // two variants timed alternately on one MI355X): N = 65536 at 16 items per CU with the
    // j-split bounded by the tiles only, 2.565 against 2.726 ms; 131072 at 64 items per CU,
    // 10.07 against 11.20 ms.  From 4096 to 32768 the tuner's other choices were within 3 % of
    // the defaults above once the clocks were warm, and from 262144 the defaults win.
    if (n >= 49152 && n < 98304) {
        v.target = num_cu * 16;
        v.kmax = 1 << 16;
    } else if (n >= 98304 && n < 196608) {
        v.target = num_cu * 64;
    }
    return v;
}

// Consecutive 256-byte aligned pieces of one caller-owned device allocation; with a NULL base it
// only counts the bytes (the pointers it hands out are then NULL).
struct Carver {
    char *base;
    size_t off = 0;
    template <class T>
    T *take(size_t count) {
        off = (off + 255) & ~(size_t)255;
        T *p = base ? (T *)(base + off) : nullptr;
        off += std::max<size_t>(count * sizeof(T), 16);
        return p;
    }
};

nb_status enqueue_predict(nb_ctx *c, const int64_t *t, int guard, hipStream_t s) {
    const StateView sv = state_view(c);
    const int32_t grid = grid_for(c->n, 8192);
    switch (c->prec) {
        case NB_FP32:
        case NB_FP32_FIXED: predict_kernel<0><<<grid, WG, 0, s>>>(sv, c->js, t, c->ctl, guard); break;
        case NB_DS: predict_kernel<1><<<grid, WG, 0, s>>>(sv, c->js, t, c->ctl, guard); break;
        case NB_FP32_ALL: predict_kernel<3><<<grid, WG, 0, s>>>(sv, c->js, t, c->ctl, guard); break;
        default: predict_kernel<2><<<grid, WG, 0, s>>>(sv, c->js, t, c->ctl, guard); break;
    }
    LAUNCH_OK(c);
    return NB_OK;
}

template <class M, int IPL, int UNR>
void launch_soft(const typename M::Args &pa, const ForceCommon &fc, bool soft, int cls,
                 int32_t grid, hipStream_t s) {
    if (cls == 0) {
        if (soft) force_kernel<M, IPL, UNR, true, 0><<<grid, WG, 0, s>>>(pa, fc);
        else force_kernel<M, IPL, UNR, false, 0><<<grid, WG, 0, s>>>(pa, fc);
    } else {
        if (soft) force_kernel<M, IPL, UNR, true, 1><<<grid, WG, 0, s>>>(pa, fc);
        else force_kernel<M, IPL, UNR, false, 1><<<grid, WG, 0, s>>>(pa, fc);
    }
}

template <class M>
void launch_ipl1(const typename M::Args &pa, const ForceCommon &fc, const Variant &v, bool soft,
                 int cls, int32_t grid, hipStream_t s) {
    if (v.unroll == 1) launch_soft<M, 1, 1>(pa, fc, soft, cls, grid, s);
    else launch_soft<M, 1, 2>(pa, fc, soft, cls, grid, s);
}

void launch_f32(const ModeF32::Args &pa, const ForceCommon &fc, const Variant &v, bool soft,
                int cls, int32_t grid, hipStream_t s) {
    if (v.ipl == 4) {
        if (v.unroll == 1) launch_soft<ModeF32, 4, 1>(pa, fc, soft, cls, grid, s);
        else launch_soft<ModeF32, 4, 2>(pa, fc, soft, cls, grid, s);
    } else if (v.ipl == 2) {
        if (v.unroll == 1) launch_soft<ModeF32, 2, 1>(pa, fc, soft, cls, grid, s);
        else if (v.unroll == 2) launch_soft<ModeF32, 2, 2>(pa, fc, soft, cls, grid, s);
        else launch_soft<ModeF32, 2, 4>(pa, fc, soft, cls, grid, s);
    } else {
        if (v.unroll == 1) launch_soft<ModeF32, 1, 1>(pa, fc, soft, cls, grid, s);
        else if (v.unroll == 2) launch_soft<ModeF32, 1, 2>(pa, fc, soft, cls, grid, s);
        else launch_soft<ModeF32, 1, 4>(pa, fc, soft, cls, grid, s);
    }
}

void launch_fixed(const ModeF32Fixed::Args &pa, const ForceCommon &fc, const Variant &v,
                  bool soft, int cls, int32_t grid, hipStream_t s) {
    if (v.ipl == 2) {
        if (v.unroll == 1) launch_soft<ModeF32Fixed, 2, 1>(pa, fc, soft, cls, grid, s);
        else launch_soft<ModeF32Fixed, 2, 2>(pa, fc, soft, cls, grid, s);
    } else {
        if (v.unroll == 1) launch_soft<ModeF32Fixed, 1, 1>(pa, fc, soft, cls, grid, s);
        else launch_soft<ModeF32Fixed, 1, 2>(pa, fc, soft, cls, grid, s);
    }
}

// Largest lane split of a precision's force kernel (fixed-point sums: whole 64-j sub-blocks).
int32_t smax_of(int prec) { return prec == NB_FP32_FIXED ? TJ / ModeTraits<ModeF32Fixed>::FOLD : 64; }

// Largest K * P over every i-count up to n_i_max against n j-particles, for one variant (the
// plan depends on the count only through its number of i-blocks, and lists shorter than a
// workgroup have the one i-block's K with fewer rows).
int64_t partial_rows_upto(int32_t n_i_max, int32_t n, const Variant &v, int32_t smax) {
    const int32_t ib = WG * v.ipl;
    int64_t rows = 0;
    for (int32_t nb = 1; nb <= (n_i_max + ib - 1) / ib; ++nb) {
        const ForcePlan pl = make_plan((int32_t)std::min<int64_t>((int64_t)nb * ib, n_i_max), n,
                                       ib, v.target, v.kmax, smax);
        if (pl.K > 1) rows = std::max<int64_t>(rows, (int64_t)pl.K * pl.P);
        if (pl.K == 1) break;  // K only falls as the number of i-blocks grows
    }
    return rows;
}

// Largest K * P over every i-count up to n, for one variant.
int64_t partial_rows_for(int32_t n, const Variant &v, int32_t smax) {
    return partial_rows_upto(n, n, v, smax);
}

// partial: the j-split partial planes (NULL: the context's own, in its workspace).
nb_status enqueue_force(nb_ctx *c, const Variant &v, int cls, const int32_t *ilist,
                        const int32_t *n_i_dev, int32_t n_i_max, double *acc, double *jerk,
                        double *pot, int32_t ld, hipStream_t s, double *partial = nullptr,
                        bool second_pass = true) {
    const int32_t ib = WG * v.ipl;
    const int32_t smax = smax_of(c->prec);
    ForceCommon fc{c->n, ilist, n_i_dev, n_i_max, v.target, v.kmax, acc, jerk, pot, ld,
                   partial ? partial : c->partial, c->ctl, smax, v.scalar_tiles};
    int32_t grid;
    if (n_i_dev) {
        // the count is known only on the device: enough workgroups for any count up to n_i_max
        const ForcePlan full = make_plan(n_i_max, c->n, ib, v.target, v.kmax, smax);
        grid = std::max(std::max(1, v.target), std::min(full.items, 65535));
    } else {
        const ForcePlan p = make_plan(n_i_max, c->n, ib, v.target, v.kmax, smax);
        grid = std::min(p.items, 1 << 20);
    }
    grid = (grid + 7) & ~7;  // a multiple of 8: the force kernel's XCD-aware item order
    const bool soft = c->eps > 0.0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->profile) {
        HIP_OK(c, hipEventCreate(&e0));
        HIP_OK(c, hipEventCreate(&e1));
        HIP_OK(c, hipEventRecord(e0, s));
    }
    switch (c->prec) {
        case NB_FP32: {
            ModeF32::Args pa{c->js.px, c->js.py, c->js.pz, c->js.vm, (float)(c->eps * c->eps)};
            launch_f32(pa, fc, v, soft, cls, grid, s);
            break;
        }
        case NB_FP32_FIXED: {
            ModeF32Fixed::Args pa{c->js.px, c->js.py, c->js.pz, c->js.vm, (float)(c->eps * c->eps)};
            launch_fixed(pa, fc, v, soft, cls, grid, s);
            break;
        }
        case NB_FP32_ALL: {
            ModeF32All::Args pa{c->js.q0, c->js.q1, (float)(c->eps * c->eps)};
            launch_ipl1<ModeF32All>(pa, fc, v, soft, cls, grid, s);
            break;
        }
        case NB_DS: {
            const double e2 = c->eps * c->eps;
            const float h = (float)e2;
            ModeDS::Args pa{c->js.q0, c->js.q1, c->js.q2, c->js.q3, ds{h, (float)(e2 - (double)h)}};
            launch_ipl1<ModeDS>(pa, fc, v, soft, cls, grid, s);
            break;
        }
        default: {
            ModeF64::Args pa{c->js.px, c->js.py, c->js.pz, c->js.pm, c->js.vx, c->js.vy, c->js.vz,
                             c->eps * c->eps};
            launch_ipl1<ModeF64>(pa, fc, v, soft, cls, grid, s);
            break;
        }
    }
    LAUNCH_OK(c);
    if (c->profile) {
        HIP_OK(c, hipEventRecord(e1, s));
        c->ev.push_back(nb_ctx::Timed{e0, e1, cls});
    }
    if (!second_pass) return NB_OK;  // the caller sums the partials (reduce_correct_level)
    // second pass: a no-op when the plan has K == 1
    const int32_t units = ((n_i_max + 63) / 64) * 7;
    const int32_t rgrid = std::max(1, std::min(units, c->num_cu * 8));
    if (c->prec == NB_FP32_FIXED) force_reduce<true><<<rgrid, WG_REDUCE, 0, s>>>(fc, ib);
    else force_reduce<false><<<rgrid, WG_REDUCE, 0, s>>>(fc, ib);
    LAUNCH_OK(c);
    return NB_OK;
}

nb_status enqueue_schedule(nb_ctx *c, double eta, hipStream_t s) {
    const StateRW rw = state_rw(c);
    sched_newlevel<<<grid_for(c->n, 2048), WG, 0, s>>>(rw, c->active, c->crit, eta, c->lmin,
                                                        c->lmax, c->ctl);
    LAUNCH_OK(c);
    const SchedView sv = sched_view(c);
    sched_min<<<c->sched_groups, WG, 0, s>>>(sv);
    LAUNCH_OK(c);
    sched_count<<<c->sched_groups, WG, 0, s>>>(sv, c->ctl);
    LAUNCH_OK(c);
    sched_scatter<<<c->sched_groups, WG, 0, s>>>(sv, c->ctl);
    LAUNCH_OK(c);
    return NB_OK;
}

nb_status enqueue_correct(nb_ctx *c, const double *acc, const double *jerk, const double *pot,
                          hipStream_t s) {
    correct_kernel<<<grid_for(c->n, 2048), WG, 0, s>>>(state_rw(c), c->active, acc, jerk, pot,
                                                        c->n, c->crit, c->ctl);
    LAUNCH_OK(c);
    return NB_OK;
}

// Before fused steps: new levels for a block left corrected by a separate nb_correct, then the
// per-level histogram rebuilt from the bound state (levels may have been set by any call).
nb_status enqueue_fused_prelude(nb_ctx *c, double eta, hipStream_t s) {
    sched_newlevel<<<grid_for(c->n, 2048), WG, 0, s>>>(state_rw(c), c->active, c->crit, eta, c->lmin,
                                                        c->lmax, c->ctl);
    LAUNCH_OK(c);
    hist_clear<<<1, WG, 0, s>>>(c->ctl);
    LAUNCH_OK(c);
    hist_build<<<grid_for(c->n, 2048), WG, 0, s>>>(c->st.level, c->n, c->ctl);
    LAUNCH_OK(c);
    return NB_OK;
}

// One block step as three launches: selection + predict, force, reduction + correct + new
// levels.
nb_status enqueue_step(nb_ctx *c, double eta, hipStream_t s) {
    nb_status r;
    const StateView sv = state_view(c);
    const SchedView fv = fused_view(c);
    const int32_t g = c->fused_groups;
    switch (c->prec) {
        case NB_FP32:
        case NB_FP32_FIXED: fused_select_predict<0><<<g, WG, 0, s>>>(fv, sv, c->js, c->ctl); break;
        case NB_DS: fused_select_predict<1><<<g, WG, 0, s>>>(fv, sv, c->js, c->ctl); break;
        case NB_FP32_ALL: fused_select_predict<3><<<g, WG, 0, s>>>(fv, sv, c->js, c->ctl); break;
        default: fused_select_predict<2><<<g, WG, 0, s>>>(fv, sv, c->js, c->ctl); break;
    }
    LAUNCH_OK(c);
    if ((r = enqueue_force(c, c->var_block, 1, c->active, &c->ctl->n_act, c->n, c->acc1, c->jerk1,
                           c->pot1, c->n, s, nullptr, false)) != NB_OK)
        return r;
    // the j-split sums and the corrector in one launch; the same ForceCommon as the force
    const Variant &v = c->var_block;
    ForceCommon fc{c->n, c->active, &c->ctl->n_act, c->n, v.target, v.kmax, c->acc1, c->jerk1,
                   c->pot1, c->n, c->partial, c->ctl, smax_of(c->prec), v.scalar_tiles};
    const int32_t units = (c->n + RC_ROWS - 1) / RC_ROWS;
    const int32_t rgrid = (std::max(8, std::min(units, c->num_cu * 2)) + 7) & ~7;
    if (c->prec == NB_FP32_FIXED)
        reduce_correct_level<true><<<rgrid, WG_REDUCE, 0, s>>>(fc, WG * v.ipl, state_rw(c), eta,
                                                                c->lmin, c->lmax, c->ctl);
    else
        reduce_correct_level<false><<<rgrid, WG_REDUCE, 0, s>>>(fc, WG * v.ipl, state_rw(c), eta,
                                                                 c->lmin, c->lmax, c->ctl);
    LAUNCH_OK(c);
    return NB_OK;
}

// nb_run's resident path: contexts of at most resident_max softened particles in the FP32,
// double-single or FP64 arithmetic.
bool use_resident(const nb_ctx *c) {
    return c->n <= c->resident_max && c->n <= RES_MAX && c->eps > 0.0 &&
           (c->prec == NB_FP32 || c->prec == NB_DS || c->prec == NB_FP64);
}

nb_status enqueue_resident(nb_ctx *c, double eta, int32_t steps, hipStream_t s) {
    const StateRW rw = state_rw(c);
    const double e2 = c->eps * c->eps;
    switch (c->prec) {
        case NB_FP32:
            run_resident<ModeF32><<<1, WGL, 0, s>>>(rw, c->active, c->ctl, e2, eta, c->lmin, c->lmax,
                                                    steps);
            break;
        case NB_DS:
            run_resident<ModeDS><<<1, WGL, 0, s>>>(rw, c->active, c->ctl, e2, eta, c->lmin, c->lmax,
                                                   steps);
            break;
        default:
            run_resident<ModeF64><<<1, WGL, 0, s>>>(rw, c->active, c->ctl, e2, eta, c->lmin, c->lmax,
                                                    steps);
            break;
    }
    LAUNCH_OK(c);
    return NB_OK;
}

nb_status latched(nb_ctx *c) {
    DevControl h;
    HIP_OK(c, hipMemcpyAsync(&h, c->ctl, sizeof h, hipMemcpyDeviceToHost, c->stream));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    if (h.flag_nonfinite) return fail(c, NB_ENONFINITE, "non-finite force or state on device");
    if (h.flag_sched)
        return fail(c, NB_ESTATE, "block selection: a particle's next time preceded the block time");
    if (h.flag_dtmin) return fail(c, NB_EDTMIN, "time step below 2^-%d requested (clamped)", c->lmax);
    return NB_OK;
}

void drop_graph(nb_ctx *c) {
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->gexec = nullptr;
    c->graph = nullptr;
    c->graph_steps = 0;
}

bool ctx_args_ok(int32_t n, int32_t precision) {
    return n >= 1 && n <= (1 << 28) && precision >= NB_FP32 && precision <= NB_FP32_FIXED;
}

int device_cus(int device) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        return prop.multiProcessorCount;
    return 256;
}

// Launch defaults and the sizes of the work buffers, from n, the precision and the CU count.
void ctx_plan(nb_ctx *c) {
    const int32_t n = c->n, precision = c->prec;
    c->var_full = default_variant(n, precision, c->num_cu, false);
    c->var_block = default_variant(n, precision, c->num_cu, true);
    c->max_target = c->num_cu * FULL_ITEMS_PER_CU;
    // partial planes: K * P rows for the largest plan of either target family, one or two i
    // per work-item, for any count up to n (variant_valid refuses a variant, e.g. four i per
    // work-item at a large target, whose plan would need more)
    int64_t rows = 0;
    for (int ipl = 1; ipl <= 2; ++ipl) {
        // two i per work-item: sized for half the full target (the same partial rows); the
        // scalar-load threshold does not change the plan
        rows = std::max(rows, partial_rows_for(n, Variant{ipl, 1, c->num_cu * FULL_ITEMS_PER_CU / ipl,
                                                          FULL_KMAX, 1}, smax_of(precision)));
        rows = std::max(rows, partial_rows_for(n, Variant{ipl, 1, c->num_cu * BLOCK_ITEMS_PER_CU,
                                                          1 << 16, 1}, smax_of(precision)));
    }
    // the force VJP writes K * P rows of its plan even when K = 1
    {
        const ForcePlan pv = make_plan(n, n, WG, c->num_cu * BLOCK_ITEMS_PER_CU, 1 << 16);
        rows = std::max<int64_t>(rows, (int64_t)pv.K * pv.P);
    }
    c->partial_rows = rows;
    const int64_t N = n;
    c->sched_groups = (int32_t)std::min<int64_t>(std::max<int64_t>((N + 4095) / 4096, 1), 1024);
    c->sched_chunk = (int32_t)((N + c->sched_groups - 1) / c->sched_groups);
    // the fused step predicts while it counts: chunks of 256 up to N = 65536 (at least one
    // workgroup per compute unit there; against chunks of 1024, alternated on one MI355X: the
    // N = 65536 run 2.744 against 2.805 s, block steps at N = 2048 - 32768 5 - 10 % shorter),
    // chunks of 1024 above (within 1 % either way from N = 131072), up to 2048 chunks
    c->fused_groups = N <= 65536
        ? (int32_t)std::max<int64_t>((N + 255) / 256, 1)
        : (int32_t)std::min<int64_t>((N + 1023) / 1024, 2048);
    c->fused_chunk = (int32_t)((N + c->fused_groups - 1) / c->fused_groups);
}

// Work buffers of a context in its workspace (base NULL: only the total size, returned).
//   j-particle stream   64 B per particle (the widest layout, double-single)
//   block force outputs acc, jerk (3 n each), pot (n), FP64
//   j-split partials    7 * partial_rows FP64
//   block list (n int32), criterion inputs (2 n FP64), per-workgroup minima and counts,
//   scheduler record, energy scratch (8 n + 2 FP64), adjoint scratch (12 n FP64) and flags,
//   the zero tick and the tuner's device count.
size_t ctx_layout(nb_ctx *c, char *base) {
    Carver k{base};
    const size_t N = (size_t)c->n;
    c->jbuf = k.take<char>(64 * N);
    c->js = JStreamView{};
    if (base) {
        char *b = (char *)c->jbuf;
        if (c->prec == NB_FP32 || c->prec == NB_FP32_FIXED) {
            c->js.px = (double *)b; c->js.py = c->js.px + N; c->js.pz = c->js.py + N;
            c->js.vm = (float4 *)(c->js.pz + N);
        } else if (c->prec == NB_DS) {
            c->js.q0 = (float4 *)b; c->js.q1 = c->js.q0 + N; c->js.q2 = c->js.q1 + N;
            c->js.q3 = c->js.q2 + N;
        } else if (c->prec == NB_FP32_ALL) {
            c->js.q0 = (float4 *)b; c->js.q1 = c->js.q0 + N;
        } else {
            c->js.px = (double *)b; c->js.py = c->js.px + N; c->js.pz = c->js.py + N;
            c->js.pm = c->js.pz + N; c->js.vx = c->js.pm + N; c->js.vy = c->js.vx + N;
            c->js.vz = c->js.vy + N;
        }
    }
    c->acc1 = k.take<double>(7 * N);
    c->jerk1 = base ? c->acc1 + 3 * N : nullptr;
    c->pot1 = base ? c->jerk1 + 3 * N : nullptr;
    c->partial = k.take<double>((size_t)std::max<int64_t>(c->partial_rows, 1) * 7);
    c->active = k.take<int32_t>(N);
    c->crit = k.take<double>(2 * N);
    const int32_t ngroups = std::max(c->sched_groups, c->fused_groups);
    c->wgmin = k.take<int64_t>(ngroups);
    c->cnt = k.take<int32_t>(ngroups);
    c->ctl = k.take<DevControl>(1);
    c->exp_ = k.take<double>(8 * N + 2);
    if (base) {
        c->evp = c->exp_ + 3 * N; c->ew = c->evp + 3 * N; c->ek = c->ew + N; c->eout = c->ek + N;
    }
    c->adj = k.take<double>(12 * N);
    c->adj_flag = k.take<int32_t>(4);
    c->t_zero = k.take<int64_t>(1);
    c->tune_n = k.take<int32_t>(1);
    return k.off;
}

nb_status need(nb_ctx *c, bool bound_required = true) {
    if (!c) return NB_EINVAL;
    if (!c->scratch_ok)
        return fail(c, NB_ESTATE, "no workspace bound (call nb_bind_scratch)");
    if (bound_required && !c->bound) return fail(c, NB_ESTATE, "state not bound (call nb_bind)");
    HIP_OK(c, hipSetDevice(c->device));
    return NB_OK;
}

}  // namespace

extern "C" {

const char *nb_version(void) { return "libnbody 0.1 gfx950"; }

const char *nb_last_error(const nb_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

nb_status nb_create(nb_ctx **out, int32_t n, double eps, int32_t lmin, int32_t lmax,
                    int32_t precision) {
    if (!out) return NB_EINVAL;
    *out = nullptr;
    if (!ctx_args_ok(n, precision) || !(eps >= 0.0) || !std::isfinite(eps) || lmin < 0 ||
        lmax < lmin || lmax > 52)
        return NB_EINVAL;
    nb_ctx *c = new nb_ctx();
    c->n = n; c->eps = eps; c->lmin = lmin; c->lmax = lmax; c->prec = precision;
    if (hipGetDevice(&c->device) != hipSuccess) { delete c; return NB_EDEVICE; }
    c->num_cu = device_cus(c->device);
    noalloc_setup(c->device);
    ctx_plan(c);
    c->scratch_need = ctx_layout(c, nullptr);
    if (hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        return NB_EDEVICE;
    }
    *out = c;
    return NB_OK;
}

size_t nb_scratch_bytes(int32_t n, int32_t precision) {
    if (!ctx_args_ok(n, precision)) return 0;
    int dev = 0;
    nb_ctx c;
    c.n = n; c.prec = precision;
    c.num_cu = hipGetDevice(&dev) == hipSuccess ? device_cus(dev) : 256;  // no device: MI355X
    ctx_plan(&c);
    return ctx_layout(&c, nullptr);
}

nb_status nb_bind_scratch(nb_ctx *c, void *scratch, size_t bytes) {
    if (!c) return NB_EINVAL;
    if (!scratch) return fail(c, NB_EINVAL, "nb_bind_scratch: workspace pointer required");
    if ((uintptr_t)scratch % 256 != 0)
        return fail(c, NB_EINVAL, "nb_bind_scratch: workspace must be 256-byte aligned");
    if (bytes < c->scratch_need)
        return fail(c, NB_EINVAL, "nb_bind_scratch: %zu bytes given, %zu needed", bytes,
                    c->scratch_need);
    HIP_OK(c, hipSetDevice(c->device));
    if (c->stream) HIP_OK(c, hipStreamSynchronize(c->stream));
    drop_graph(c);
    ctx_layout(c, (char *)scratch);
    zero_words<<<1, WG, 0, c->stream>>>(c->t_zero, 2, c->adj_flag, 4);
    LAUNCH_OK(c);
    reset_control<<<1, WG, 0, c->stream>>>(c->ctl);
    LAUNCH_OK(c);
    c->scratch_ok = true;
    c->predicted = false;
    c->forced = false;
    return NB_OK;
}

nb_status nb_destroy(nb_ctx *c) {
    if (!c) return NB_OK;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    (void)hipDeviceSynchronize();
    drop_graph(c);
    for (auto &p : c->ev) {
        (void)hipEventDestroy(p.start);
        (void)hipEventDestroy(p.stop);
    }
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    delete c;
    return NB_OK;
}

nb_status nb_set_stream(nb_ctx *c, void *stream) {
    if (!c) return NB_EINVAL;
    c->stream = (hipStream_t)stream;
    return NB_OK;
}

nb_status nb_bind(nb_ctx *c, const nb_state *s) {
    if (!c || !s) return NB_EINVAL;
    if (!s->x || !s->v || !s->a || !s->k || !s->m || !s->pot || !s->tick || !s->level)
        return fail(c, NB_EINVAL, "nb_bind: every state array is required");
    c->st = *s;
    c->bound = true;
    c->predicted = false;
    c->forced = false;
    drop_graph(c);
    return NB_OK;
}

nb_status nb_init(nb_ctx *c, double eta) {
    nb_status r;
    if ((r = need(c)) != NB_OK) return r;
    if (!(eta > 0.0) || !std::isfinite(eta)) return fail(c, NB_EINVAL, "eta must be > 0");
    hipStream_t s = c->stream;
    reset_control<<<1, WG, 0, s>>>(c->ctl);
    LAUNCH_OK(c);
    zero_ticks<<<grid_for(c->n, 4096), WG, 0, s>>>(c->st.tick, c->n);
    LAUNCH_OK(c);
    if ((r = enqueue_predict(c, c->t_zero, 0, s)) != NB_OK) return r;
    if ((r = enqueue_force(c, c->var_full, 0, nullptr, nullptr, c->n, c->acc1, c->jerk1, c->pot1,
                           c->n, s)) != NB_OK)
        return r;
    init_levels<<<grid_for(c->n, 4096), WG, 0, s>>>(state_rw(c), c->acc1, c->jerk1, c->pot1, eta,
                                                      c->lmin, c->lmax, c->ctl);
    LAUNCH_OK(c);
    c->predicted = true;
    c->forced = false;
    return enqueue_schedule(c, eta, s);
}

nb_status nb_schedule_block(nb_ctx *c, double eta) {
    nb_status r;
    if ((r = need(c)) != NB_OK) return r;
    if (!(eta > 0.0) || !std::isfinite(eta)) return fail(c, NB_EINVAL, "eta must be > 0");
    return enqueue_schedule(c, eta, c->stream);
}

nb_status nb_active(nb_ctx *c, const int32_t **idx, const int32_t **n_act) {
    if (!c || !idx || !n_act) return NB_EINVAL;
    if (!c->scratch_ok) return fail(c, NB_ESTATE, "no workspace bound (call nb_bind_scratch)");
    *idx = c->active;
    *n_act = &c->ctl->n_act;
    return NB_OK;
}

nb_status nb_predict(nb_ctx *c, const int64_t *t) {
    nb_status r;
    if ((r = need(c)) != NB_OK) return r;
    if ((r = enqueue_predict(c, t, 0, c->stream)) != NB_OK) return r;
    c->predicted = true;
    return NB_OK;
}

nb_status nb_force(nb_ctx *c, const int32_t *i_idx, const int32_t *n_i, int32_t n_i_max,
                   double *acc, double *jerk, double *pot) {
    nb_status r;
    if ((r = need(c)) != NB_OK) return r;
    if (!c->predicted) return fail(c, NB_ESTATE, "nb_force before nb_predict");
    if (!acc || !jerk || !pot) return fail(c, NB_EINVAL, "nb_force: output pointers required");
    if (n_i_max < 0 || n_i_max > c->n)
        return fail(c, NB_EINVAL, "nb_force: n_i_max %d outside [0, %d]", n_i_max, c->n);
    if (!i_idx && !n_i && n_i_max == 0) return NB_OK;
    const int cls = (n_i == nullptr && n_i_max > c->n / 8) ? 0 : 1;
    if ((r = enqueue_force(c, cls == 0 ? c->var_full : c->var_block, cls, i_idx, n_i, n_i_max,
                           acc, jerk, pot, n_i_max, c->stream)) != NB_OK)
        return r;
    c->forced = true;
    return NB_OK;
}

nb_status nb_force_noalloc(nb_ctx *c, const int32_t *i_idx, const int32_t *n_i,
                           int32_t n_i_max, double *acc, double *jerk, double *pot) {
    nb_status r;
    if ((r = need(c)) != NB_OK) return r;
    if (!c->predicted) return fail(c, NB_ESTATE, "nb_force_noalloc before nb_predict");
    if (!acc || !jerk || !pot) return fail(c, NB_EINVAL, "nb_force_noalloc: output pointers required");
    if (n_i_max < 0 || n_i_max > c->n)
        return fail(c, NB_EINVAL, "nb_force_noalloc: n_i_max %d outside [0, %d]", n_i_max, c->n);
    if (!i_idx && !n_i && n_i_max == 0) return NB_OK;
    const int cls = (n_i == nullptr && n_i_max > c->n / 8) ? 0 : 1;
    const Variant &v = cls == 0 ? c->var_full : c->var_block;
    const int32_t smax = smax_of(c->prec);
    // partial-sum rows of this call's plan (for a device count: of the largest count it allows)
    int64_t rows = 0;
    if (n_i) {
        rows = partial_rows_upto(n_i_max, c->n, v, smax);
    } else {
        const ForcePlan pl = make_plan(n_i_max, c->n, WG * v.ipl, v.target, v.kmax, smax);
        rows = pl.K > 1 ? (int64_t)pl.K * pl.P : 0;
    }
    const size_t bytes = (size_t)rows * 7 * sizeof(double);
    if (bytes > NOALLOC_SCRATCH_BYTES)
        return fail(c, NB_EINVAL,
                    "nb_force_noalloc: this call's j-split needs %zu bytes of partial sums; the "
                    "static array holds %zu (use nb_force)", bytes, NOALLOC_SCRATCH_BYTES);
    double *part = (double *)noalloc_scratch(c->device);
    if (!part) return fail(c, NB_EDEVICE, "nb_force_noalloc: no device address for the static array");
    if ((r = enqueue_force(c, v, cls, i_idx, n_i, n_i_max, acc, jerk, pot, n_i_max, c->stream,
                           part)) != NB_OK)
        return r;
    c->forced = true;
    return NB_OK;
}

nb_status nb_correct(nb_ctx *c, const double *acc, const double *jerk, const double *pot) {
    nb_status r;
    if ((r = need(c)) != NB_OK) return r;
    if (!acc || !jerk || !pot) return fail(c, NB_EINVAL, "nb_correct: force arrays required");
    return enqueue_correct(c, acc, jerk, pot, c->stream);
}

nb_status nb_step(nb_ctx *c, double eta, int32_t nsteps, int32_t use_graph) {
    nb_status r;
    if ((r = need(c)) != NB_OK) return r;
    if (!(eta > 0.0) || !std::isfinite(eta)) return fail(c, NB_EINVAL, "eta must be > 0");
    if (nsteps < 0) return fail(c, NB_EINVAL, "nsteps < 0");
    if (nsteps == 0) return NB_OK;
    if ((r = enqueue_fused_prelude(c, eta, c->stream)) != NB_OK) return r;
    if (!use_graph || c->profile) {  // timing events are recorded on eager launches only
        for (int32_t i = 0; i < nsteps; ++i)
            if ((r = enqueue_step(c, eta, c->stream)) != NB_OK) return r;
        c->predicted = true;
        return NB_OK;
    }
    // One captured step, replayed nsteps times (kernel arguments bake in eta).
    if (!c->gexec || c->graph_eta != eta) {
        drop_graph(c);
        HIP_OK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
        nb_status rs = enqueue_step(c, eta, c->cap_stream);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
        if (rs != NB_OK) { if (g) (void)hipGraphDestroy(g); return rs; }
        if (e != hipSuccess) return fail(c, NB_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
        c->graph = g;
        HIP_OK(c, hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
        c->graph_eta = eta;
        c->graph_steps = 1;
    }
    for (int32_t i = 0; i < nsteps; ++i) HIP_OK(c, hipGraphLaunch(c->gexec, c->stream));
    c->predicted = true;
    return NB_OK;
}

nb_status nb_run(nb_ctx *c, double eta, int64_t t_end, int64_t max_steps, int32_t chunk,
                 int32_t use_graph) {
    nb_status r;
    if ((r = need(c)) != NB_OK) return r;
    if (chunk < 1) return fail(c, NB_EINVAL, "chunk must be >= 1");
    if (!(eta > 0.0) || !std::isfinite(eta)) return fail(c, NB_EINVAL, "eta must be > 0");
    set_t_end<<<1, WG, 0, c->stream>>>(c->ctl, t_end);
    LAUNCH_OK(c);
    const bool resident = use_resident(c) && !c->profile;
    if (resident) {  // new levels of a block corrected by a separate nb_correct
        sched_newlevel<<<grid_for(c->n, 2048), WG, 0, c->stream>>>(state_rw(c), c->active, c->crit,
                                                                    eta, c->lmin, c->lmax, c->ctl);
        LAUNCH_OK(c);
    }
    int64_t done_steps = 0;
    for (;;) {
        int32_t k = chunk;
        if (max_steps > 0) k = (int32_t)std::min<int64_t>(k, max_steps - done_steps);
        if (k <= 0) break;
        if (resident) {
            if ((r = enqueue_resident(c, eta, k, c->stream)) != NB_OK) return r;
            c->predicted = false;  // the j-particle stream was not written
        } else if ((r = nb_step(c, eta, k, use_graph)) != NB_OK) {
            return r;
        }
        done_steps += k;
        DevControl h;
        HIP_OK(c, hipMemcpyAsync(&h, c->ctl, sizeof h, hipMemcpyDeviceToHost, c->stream));
        HIP_OK(c, hipStreamSynchronize(c->stream));
        if (h.flag_nonfinite) return fail(c, NB_ENONFINITE, "non-finite force or state on device");
        if (h.done) break;
    }
    // leave the scheduler open-ended again
    set_t_end<<<1, WG, 0, c->stream>>>(c->ctl, INT64_MAX);
    LAUNCH_OK(c);
    return latched(c);
}

nb_status nb_energy(nb_ctx *c, double *ekin, double *epot) {
    nb_status r;
    if ((r = need(c)) != NB_OK) return r;
    if (!ekin || !epot) return fail(c, NB_EINVAL, "nb_energy: host outputs required");
    hipStream_t s = c->stream;
    energy_predict<<<grid_for(c->n, 8192), WG, 0, s>>>(state_view(c), c->ctl, c->exp_, c->evp);
    LAUNCH_OK(c);
    energy_pairs<<<grid_for(c->n, 1 << 20), WG, 0, s>>>(c->exp_, c->evp, c->st.m, c->n,
                                                         c->eps * c->eps, c->ew, c->ek);
    LAUNCH_OK(c);
    energy_reduce<<<1, 1024, 0, s>>>(c->ew, c->ek, c->n, c->eout);
    LAUNCH_OK(c);
    double h[2];
    HIP_OK(c, hipMemcpyAsync(h, c->eout, sizeof h, hipMemcpyDeviceToHost, s));
    HIP_OK(c, hipStreamSynchronize(s));
    *ekin = h[0];
    *epot = h[1];
    return latched(c);
}

nb_status nb_read_control(nb_ctx *c, nb_control *out) {
    if (!c || !out) return NB_EINVAL;
    if (!c->scratch_ok) return fail(c, NB_ESTATE, "no workspace bound (call nb_bind_scratch)");
    HIP_OK(c, hipSetDevice(c->device));
    DevControl h;
    HIP_OK(c, hipMemcpyAsync(&h, c->ctl, sizeof h, hipMemcpyDeviceToHost, c->stream));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    out->t_cur = h.t_cur; out->t_next = h.t_next; out->t_end = h.t_end;
    out->n_steps = h.n_steps; out->n_active_sum = h.n_active_sum; out->n_act = h.n_act;
    out->flags = (h.flag_nonfinite ? 1 : 0) | (h.flag_dtmin ? 2 : 0) | (h.flag_sched ? 4 : 0);
    if (h.flag_nonfinite) return fail(c, NB_ENONFINITE, "non-finite force or state on device");
    if (h.flag_sched)
        return fail(c, NB_ESTATE, "block selection: a particle's next time preceded the block time");
    if (h.flag_dtmin) return fail(c, NB_EDTMIN, "time step below 2^-%d requested (clamped)", c->lmax);
    return NB_OK;
}

static nb_status check_shared_dt(nb_ctx *c, double dt, int64_t *dt_ticks) {
    int e = 0;
    const double f = std::frexp(dt, &e);  // dt = f 2^e, f in [0.5, 1)
    const int l = 1 - e;                  // dt = 2^-l when f == 0.5
    if (!(dt > 0.0) || f != 0.5 || l < c->lmin || l > c->lmax)
        return fail(c, NB_EINVAL, "shared step dt must be 2^-l with %d <= l <= %d", c->lmin, c->lmax);
    *dt_ticks = (int64_t)1 << (c->lmax - l);
    return NB_OK;
}

static nb_status enqueue_force_vjp(nb_ctx *c, const double *ab, const double *kb, double *xb,
                                   double *vb, double *mb, int32_t accumulate, hipStream_t s) {
    VjpArgs a;
    a.n = c->n;
    a.px = c->js.px; a.py = c->js.py; a.pz = c->js.pz; a.vm = c->js.vm;
    a.pm = c->js.pm; a.vx = c->js.vx; a.vy = c->js.vy; a.vz = c->js.vz;
    a.ab = ab; a.kb = kb; a.eps2 = c->eps * c->eps; a.partial = c->partial;
    a.target = c->num_cu * BLOCK_ITEMS_PER_CU; a.kmax = 1 << 16;
    const ForcePlan pl = make_plan(c->n, c->n, WG, a.target, a.kmax);
    if ((int64_t)pl.K * pl.P > c->partial_rows)  // the workspace is sized for this plan
        return fail(c, NB_ESTATE, "force VJP plan exceeds the partial planes");
    const int32_t grid = std::max(1, std::min(pl.items, 1 << 20));
    // softened: every separation is positive in the arithmetic type, only the self pair masked
    const bool soft = c->prec == NB_FP32 ? (float)a.eps2 > 0.0f : a.eps2 > 0.0;
    if (c->prec == NB_FP32) {
        if (soft) force_vjp_kernel<0, true><<<grid, WG, 0, s>>>(a);
        else force_vjp_kernel<0, false><<<grid, WG, 0, s>>>(a);
    } else {
        if (soft) force_vjp_kernel<2, true><<<grid, WG, 0, s>>>(a);
        else force_vjp_kernel<2, false><<<grid, WG, 0, s>>>(a);
    }
    LAUNCH_OK(c);
    vjp_reduce<<<grid_for(c->n, 4096), WG, 0, s>>>(c->n, c->partial, a.target, a.kmax, xb, vb, mb,
                                                   accumulate);
    LAUNCH_OK(c);
    return NB_OK;
}

static nb_status enqueue_shared_predict(nb_ctx *c, double dt, hipStream_t s) {
    const int32_t grid = grid_for(c->n, 8192);
    if (c->prec == NB_FP32) shared_predict<0><<<grid, WG, 0, s>>>(state_view(c), c->js, dt);
    else shared_predict<2><<<grid, WG, 0, s>>>(state_view(c), c->js, dt);
    LAUNCH_OK(c);
    return NB_OK;
}

nb_status nb_shared_step(nb_ctx *c, double dt, int32_t nsteps) {
    nb_status r;
    if ((r = need(c)) != NB_OK) return r;
    if (c->prec != NB_FP32 && c->prec != NB_FP64)
        return fail(c, NB_EINVAL, "shared steps: fp32 or fp64 contexts only");
    int64_t dt_ticks = 0;
    if ((r = check_shared_dt(c, dt, &dt_ticks)) != NB_OK) return r;
    if (nsteps < 0) return fail(c, NB_EINVAL, "nsteps < 0");
    hipStream_t s = c->stream;
    for (int32_t k = 0; k < nsteps; ++k) {
        if ((r = enqueue_shared_predict(c, dt, s)) != NB_OK) return r;
        if ((r = enqueue_force(c, c->var_full, 0, nullptr, nullptr, c->n, c->acc1, c->jerk1,
                               c->pot1, c->n, s)) != NB_OK)
            return r;
        shared_correct<<<grid_for(c->n, 8192), WG, 0, s>>>(state_rw(c), c->acc1, c->jerk1,
                                                           c->pot1, dt, dt_ticks, c->adj_flag);
        LAUNCH_OK(c);
    }
    c->predicted = true;
    return NB_OK;
}

nb_status nb_force_vjp(nb_ctx *c, const double *abar, const double *kbar, double *xbar,
                       double *vbar, double *mbar) {
    nb_status r;
    if ((r = need(c)) != NB_OK) return r;
    if (c->prec != NB_FP32 && c->prec != NB_FP64)
        return fail(c, NB_EINVAL, "force VJP: fp32 or fp64 contexts only");
    if (!c->predicted) return fail(c, NB_ESTATE, "nb_force_vjp before nb_predict");
    if (!abar || !kbar || !xbar || !vbar || !mbar) return fail(c, NB_EINVAL, "nb_force_vjp: arrays required");
    return enqueue_force_vjp(c, abar, kbar, xbar, vbar, mbar, 1, c->stream);
}

nb_status nb_step_vjp(nb_ctx *c, double dt, double *xbar, double *vbar, double *abar,
                      double *kbar, double *mbar) {
    nb_status r;
    if ((r = need(c)) != NB_OK) return r;
    if (c->prec != NB_FP32 && c->prec != NB_FP64)
        return fail(c, NB_EINVAL, "step VJP: fp32 or fp64 contexts only");
    int64_t dt_ticks = 0;
    if ((r = check_shared_dt(c, dt, &dt_ticks)) != NB_OK) return r;
    if (!xbar || !vbar || !abar || !kbar || !mbar) return fail(c, NB_EINVAL, "nb_step_vjp: arrays required");
    hipStream_t s = c->stream;
    const int64_t N3 = 3 * (int64_t)c->n;
    double *a1b = c->adj, *k1b = a1b + N3, *xpb = k1b + N3, *vpb = xpb + N3;
    const int32_t g = grid_for(N3, 8192);
    if ((r = enqueue_shared_predict(c, dt, s)) != NB_OK) return r;
    vjp_pre<<<g, WG, 0, s>>>(c->n, dt, xbar, vbar, abar, kbar, a1b, k1b);
    LAUNCH_OK(c);
    if ((r = enqueue_force_vjp(c, a1b, k1b, xpb, vpb, mbar, 0, s)) != NB_OK) return r;
    vjp_post<<<g, WG, 0, s>>>(c->n, dt, xbar, vbar, abar, kbar, xpb, vpb);
    LAUNCH_OK(c);
    c->predicted = true;
    return NB_OK;
}

static bool variant_valid(const nb_ctx *c, const nb_variant &v) {
    if (!variant_compiled(c->prec, v)) return false;
    if (v.target < 1 || v.target > c->max_target || v.kmax < 1 || v.kmax > (1 << 16)) return false;
    if (v.scalar_tiles < 1 || v.scalar_tiles > (1 << 16)) return false;
    return partial_rows_for(c->n, v, smax_of(c->prec)) <= c->partial_rows;
}

nb_status nb_get_variant(nb_ctx *c, int32_t which, nb_variant *out) {
    if (!c || !out || which < 0 || which > 1) return NB_EINVAL;
    *out = which == 0 ? c->var_full : c->var_block;
    return NB_OK;
}

nb_status nb_set_variant(nb_ctx *c, int32_t which, const nb_variant *vin) {
    if (!c || !vin || which < 0 || which > 1) return NB_EINVAL;
    Variant &cur = which == 0 ? c->var_full : c->var_block;
    nb_variant vv = *vin;
    if (vv.scalar_tiles == 0) vv.scalar_tiles = cur.scalar_tiles;  // keep the current value
    const nb_variant *v = &vv;
    if (!variant_valid(c, *v))
        return fail(c, NB_EINVAL,
                    "variant ipl=%d unroll=%d target=%d kmax=%d scalar_tiles=%d not available",
                    v->ipl, v->unroll, v->target, v->kmax, v->scalar_tiles);
    cur = *v;
    drop_graph(c);
    return NB_OK;
}

nb_status nb_tune(nb_ctx *c, int32_t which, int32_t n_i, int32_t reps, nb_variant *best,
                  double *best_ms) {
    nb_status r;
    if ((r = need(c)) != NB_OK) return r;
    if (which < 0 || which > 1 || n_i < 1 || n_i > c->n || reps < 1)
        return fail(c, NB_EINVAL, "nb_tune: bad arguments");
    if (!c->predicted) return fail(c, NB_ESTATE, "nb_tune before nb_predict");
    hipStream_t s = c->stream;
    HIP_OK(c, hipMemcpyAsync(c->tune_n, &n_i, sizeof n_i, hipMemcpyHostToDevice, s));
    const bool was_profiling = c->profile;
    c->profile = false;
    hipEvent_t e0, e1;
    HIP_OK(c, hipEventCreate(&e0));
    HIP_OK(c, hipEventCreate(&e1));
    nb_variant bestv = which == 0 ? c->var_full : c->var_block;
    double bms = 1e300;
    // warm the clocks first (at least 100 ms of the current variant, at most 2000 launches):
    // timed from a cold start, the first variants of the sweep would run at a lower clock
    {
        float warm = 0.f;
        for (int i = 0; i < 2000 && warm < 100.f; ++i) {
            HIP_OK(c, hipEventRecord(e0, s));
            if (which == 0)
                r = enqueue_force(c, bestv, 0, nullptr, nullptr, n_i, c->acc1, c->jerk1, c->pot1,
                                  c->n, s);
            else
                r = enqueue_force(c, bestv, 1, nullptr, c->tune_n, c->n, c->acc1, c->jerk1,
                                  c->pot1, c->n, s);
            if (r != NB_OK) { c->profile = was_profiling; return r; }
            HIP_OK(c, hipEventRecord(e1, s));
            HIP_OK(c, hipEventSynchronize(e1));
            float ms = 0.f;
            HIP_OK(c, hipEventElapsedTime(&ms, e0, e1));
            warm += ms;
        }
    }
    const int ipls[] = {1, 2, 4}, unrs[] = {1, 2, 4}, scal[] = {1, 4, 16};
    const int32_t targets[] = {c->num_cu * 4, c->num_cu * 8, c->num_cu * 16, c->num_cu * 32,
                               c->num_cu * 64, c->num_cu * 128, c->num_cu * FULL_ITEMS_PER_CU};
    // the scalar-load threshold matters only in the float modes (FP64 always stages LDS tiles)
    const int nscal = (c->prec == NB_FP64) ? 1 : 3;
    const int32_t keep_scal = bestv.scalar_tiles;
    for (int ipl : ipls)
        for (int unr : unrs)
            for (int32_t tg : targets)
                for (int si = 0; si < nscal; ++si) {
                    const nb_variant v{ipl, unr, tg,
                                       tg > c->num_cu * BLOCK_ITEMS_PER_CU ? FULL_KMAX : 1 << 16,
                                       nscal == 1 ? keep_scal : scal[si]};
                    if (!variant_valid(c, v)) continue;
                    float tot = 0.f;
                    for (int rep = 0; rep <= reps; ++rep) {  // the first launch is not timed
                        HIP_OK(c, hipEventRecord(e0, s));
                        if (which == 0)
                            r = enqueue_force(c, v, 0, nullptr, nullptr, n_i, c->acc1, c->jerk1,
                                              c->pot1, c->n, s);
                        else
                            r = enqueue_force(c, v, 1, nullptr, c->tune_n, c->n, c->acc1,
                                              c->jerk1, c->pot1, c->n, s);
                        if (r != NB_OK) { c->profile = was_profiling; return r; }
                        HIP_OK(c, hipEventRecord(e1, s));
                        HIP_OK(c, hipEventSynchronize(e1));
                        float ms = 0.f;
                        HIP_OK(c, hipEventElapsedTime(&ms, e0, e1));
                        if (rep > 0) tot += ms;
                    }
                    const double avg = tot / reps;
                    if (avg < bms) { bms = avg; bestv = v; }
                }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->profile = was_profiling;
    (which == 0 ? c->var_full : c->var_block) = bestv;
    drop_graph(c);
    if (best) *best = bestv;
    if (best_ms) *best_ms = bms;
    return NB_OK;
}

nb_status nb_profile(nb_ctx *c, int32_t enable) {
    if (!c) return NB_EINVAL;
    HIP_OK(c, hipSetDevice(c->device));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    for (auto &p : c->ev) {
        (void)hipEventDestroy(p.start);
        (void)hipEventDestroy(p.stop);
    }
    c->ev.clear();
    c->profile = enable != 0;
    return NB_OK;
}

nb_status nb_profile_read(nb_ctx *c, int32_t which, double *ms_total, int64_t *launches) {
    if (!c || !ms_total || !launches || which < -1 || which > 1) return NB_EINVAL;
    HIP_OK(c, hipSetDevice(c->device));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    double tot = 0.0;
    int64_t cnt = 0;
    for (auto &p : c->ev) {
        if (which >= 0 && p.cls != which) continue;
        float ms = 0.f;
        HIP_OK(c, hipEventElapsedTime(&ms, p.start, p.stop));
        tot += ms;
        ++cnt;
    }
    *ms_total = tot;
    *launches = cnt;
    return NB_OK;
}

nb_status nb_fma_rate(nb_ctx *c, double *tflops) {
    nb_status r;
    if ((r = need(c, false)) != NB_OK) return r;
    if (!tflops) return fail(c, NB_EINVAL, "nb_fma_rate: host output required");
    hipStream_t s = c->stream;
    const int32_t iters = 8192, grid = c->num_cu * 64;
    hipEvent_t e0, e1;
    HIP_OK(c, hipEventCreate(&e0));
    HIP_OK(c, hipEventCreate(&e1));
    double best = 0.0;
    for (int rep = 0; rep < 12; ++rep) {  // both operand forms; the first two launches warm up
        HIP_OK(c, hipEventRecord(e0, s));
        if (rep & 1) fma_probe<true><<<grid, WG, 0, s>>>(iters, 1e-7f, 0.0f, (float *)c->eout);
        else fma_probe<false><<<grid, WG, 0, s>>>(iters, 1e-7f, 0.0f, (float *)c->eout);
        LAUNCH_OK(c);
        HIP_OK(c, hipEventRecord(e1, s));
        HIP_OK(c, hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_OK(c, hipEventElapsedTime(&ms, e0, e1));
        const double flop = 2.0 * FMA_CHAINS * (double)iters * grid * WG;
        if (rep > 1 && ms > 0.f) best = std::max(best, flop / (ms * 1e-3) / 1e12);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *tflops = best;
    return NB_OK;
}

nb_status nb_set_resident(nb_ctx *c, int32_t max_n) {
    if (!c) return NB_EINVAL;
    if (max_n < 0 || max_n > RES_MAX)
        return fail(c, NB_EINVAL, "nb_set_resident: max_n must lie in [0, %d]", RES_MAX);
    c->resident_max = max_n;
    return NB_OK;
}

nb_status nb_sync(nb_ctx *c) {
    if (!c) return NB_EINVAL;
    if (!c->scratch_ok) return fail(c, NB_ESTATE, "no workspace bound (call nb_bind_scratch)");
    HIP_OK(c, hipSetDevice(c->device));
    return latched(c);
}

}  // extern "C"

// ------------------------------------------------------------------------------------------
// Ensemble of independent clusters
// ------------------------------------------------------------------------------------------
namespace {

// lane < 0: every cluster; else the clusters of that lane (a slice of the order table)
EnsView ens_view(const nb_ens *e, int64_t t_end, int lane = -1) {
    EnsView v;
    v.C = e->C; v.off = e->off; v.K = e->K; v.tpi = e->tpi; v.order = e->order;
    if (lane >= 0) {
        v.C = e->lane_start_h[lane + 1] - e->lane_start_h[lane];
        v.order = e->order + e->lane_start_h[lane];
    }
    v.part_off = e->part_off;
    v.prow = e->prow; v.eps2 = e->eps2; v.cl = e->cl; v.active = e->active;
    v.partial = e->partial; v.crit = e->crit; v.flags = e->flags;
    v.lmin = e->lmin; v.lmax = e->lmax; v.tick_len = std::ldexp(1.0, -e->lmax); v.t_end = t_end;
    v.local_limit = e->local_limit; v.local_steps = e->local_steps; v.local_work = e->local_work;
    v.smin = e->smin;
    return v;
}

StateRW ens_state(const nb_ens *e) {
    return StateRW{e->st.x, e->st.v, e->st.a, e->st.k, e->st.m, e->st.pot, e->st.tick,
                   e->st.level, e->ntot, std::ldexp(1.0, -e->lmax)};
}

// K of each cluster from its tiles per item; the partial planes were sized for tpi = 1.
void ens_derive(nb_ens *e) {
    e->K_h.resize(e->C);
    int64_t items = 0;
    for (int32_t c = 0; c < e->C; ++c) {
        const int32_t n_c = e->off_h[c + 1] - e->off_h[c];
        const int32_t ntiles = (n_c + TJ - 1) / TJ;
        e->K_h[c] = (ntiles + e->tpi_h[c] - 1) / e->tpi_h[c];
        const int32_t ib = WG / e->smin;  // largest i-block of an item
        items += (int64_t)((n_c + ib - 1) / ib) * e->K_h[c];
    }
    e->grid_force = (int32_t)std::max<int64_t>(1, std::min<int64_t>(items, (int64_t)e->num_cu * 8));
}

#define EHIP_OK(ens, call)                                                                   \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail((ens), NB_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));   \
    } while (0)

#define ELAUNCH_OK(ens)                                                                      \
    do {                                                                                     \
        hipError_t e_ = hipGetLastError();                                                   \
        if (e_ != hipSuccess)                                                                \
            return fail((ens), NB_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e_)); \
    } while (0)

template <class M>
void ens_launch_force(nb_ens *e, const EnsView &v, hipStream_t s) {
    const StateRW rw = ens_state(e);
    const size_t lds = (size_t)(e->C + 1) * sizeof(int32_t);
    if (e->unroll == 1) ens_force<M, 1><<<e->grid_force, WG, lds, s>>>(v, rw);
    else ens_force<M, 2><<<e->grid_force, WG, lds, s>>>(v, rw);
}

// local = false: every block goes through ens_force (the start of a run)
nb_status ens_enqueue_local(nb_ens *e, double eta, int32_t phase, int64_t t_end, hipStream_t s,
                            bool local = true, int lane = -1) {
    EnsView v = ens_view(e, t_end, lane);
    if (!local) v.local_limit = 0;
    switch (e->prec) {
        case NB_FP32: ens_local<ModeF32><<<v.C, WGL, 0, s>>>(v, ens_state(e), eta, phase); break;
        case NB_DS: ens_local<ModeDS><<<v.C, WGL, 0, s>>>(v, ens_state(e), eta, phase); break;
        default: ens_local<ModeF64><<<v.C, WGL, 0, s>>>(v, ens_state(e), eta, phase); break;
    }
    ELAUNCH_OK(e);
    return NB_OK;
}

nb_status ens_enqueue_force(nb_ens *e, int64_t t_end, hipStream_t s, bool local = true,
                            int lane = -1) {
    EnsView v = ens_view(e, t_end, lane);
    if (!local) v.local_limit = 0;
    switch (e->prec) {
        case NB_FP32: ens_launch_force<ModeF32>(e, v, s); break;
        case NB_DS: ens_launch_force<ModeDS>(e, v, s); break;
        default: ens_launch_force<ModeF64>(e, v, s); break;
    }
    ELAUNCH_OK(e);
    return NB_OK;
}

// One global step: the force of every cluster's selected block that is not a local block,
// then one workgroup per cluster corrects it, selects the next block and advances the cluster
// by its local blocks.
nb_status ens_enqueue_step(nb_ens *e, double eta, int64_t t_end, hipStream_t s, int lane = -1) {
    nb_status r = ens_enqueue_force(e, t_end, s, true, lane);
    if (r != NB_OK) return r;
    return ens_enqueue_local(e, eta, 2, t_end, s, true, lane);
}

nb_status ens_upload_tables(nb_ens *e) {
    if (!e->scratch_ok) return NB_OK;  // uploaded when a workspace is bound
    EHIP_OK(e, hipMemcpy(e->K, e->K_h.data(), e->C * sizeof(int32_t), hipMemcpyHostToDevice));
    EHIP_OK(e, hipMemcpy(e->tpi, e->tpi_h.data(), e->C * sizeof(int32_t), hipMemcpyHostToDevice));
    return NB_OK;
}

void ens_drop_graph(nb_ens *e) {
    if (e->gexec) (void)hipGraphExecDestroy(e->gexec);
    if (e->graph) (void)hipGraphDestroy(e->graph);
    e->gexec = nullptr;
    e->graph = nullptr;
    for (int l = 0; l < ENS_MAX_LANES; ++l) {
        if (e->lane_gexec[l]) (void)hipGraphExecDestroy(e->lane_gexec[l]);
        if (e->lane_graph[l]) (void)hipGraphDestroy(e->lane_graph[l]);
        e->lane_gexec[l] = nullptr;
        e->lane_graph[l] = nullptr;
    }
    e->g_steps = 0;
}

bool ens_args_ok(int32_t n_clusters, const int32_t *offsets, int32_t precision) {
    if (n_clusters < 1 || n_clusters > 8192 || !offsets || offsets[0] != 0 ||
        precision < NB_FP32 || precision > NB_FP64)
        return false;
    for (int32_t c = 0; c < n_clusters; ++c)
        if (offsets[c + 1] <= offsets[c]) return false;
    return offsets[n_clusters] <= (1 << 28);
}

// Host tables of an ensemble (offsets, partial-plane sizes, default layout).
void ens_plan(nb_ens *e, int32_t n_clusters, const int32_t *offsets, int32_t precision) {
    e->C = n_clusters; e->ntot = offsets[n_clusters]; e->prec = precision;
    e->off_h.assign(offsets, offsets + n_clusters + 1);
    // default layout: the fewest whole tiles per item that leave each cluster at most
    // ENS_KMAX j-ranges (few partial planes for the cluster's own workgroup to sum)
    e->tpi_h.resize(n_clusters);
    for (int32_t c = 0; c < n_clusters; ++c) {
        const int32_t ntiles = (offsets[c + 1] - offsets[c] + TJ - 1) / TJ;
        e->tpi_h[c] = std::max(1, (ntiles + ENS_KMAX - 1) / ENS_KMAX);
    }
    e->prow_h.resize(n_clusters);
    e->part_off_h.resize(n_clusters + 1);
    e->part_off_h[0] = 0;
    for (int32_t c = 0; c < n_clusters; ++c) {
        const int32_t n_c = offsets[c + 1] - offsets[c];
        e->prow_h[c] = n_c;
        e->part_off_h[c + 1] = e->part_off_h[c] + (int64_t)((n_c + TJ - 1) / TJ) * 7 * n_c;
    }
    // the cluster-local kernel's workgroup order: decreasing size (ties by index)
    e->order_h.resize(n_clusters);
    for (int32_t c = 0; c < n_clusters; ++c) e->order_h[c] = c;
    std::stable_sort(e->order_h.begin(), e->order_h.end(), [&](int32_t a, int32_t b) {
        return offsets[a + 1] - offsets[a] > offsets[b + 1] - offsets[b];
    });
    e->size_order_h = e->order_h;
    e->lanes = 1;
    e->lane_start_h = {0, n_clusters};
    e->unroll = 2;
    ens_derive(e);
}

// Device buffers of an ensemble in its workspace (base NULL: only the total size): the cluster
// tables, per-cluster records, block lists (one slot per particle), flags, the partial planes
// (sized for one tile per work item, the finest split), criterion and energy scratch.
size_t ens_layout(nb_ens *e, char *base) {
    Carver k{base};
    const size_t C = (size_t)e->C, N = (size_t)e->ntot;
    e->off = k.take<int32_t>(C + 1);
    e->K = k.take<int32_t>(C);
    e->tpi = k.take<int32_t>(C);
    e->prow = k.take<int32_t>(C);
    e->order = k.take<int32_t>(C);
    e->part_off = k.take<int64_t>(C + 1);
    e->eps2 = k.take<double>(C);
    e->cl = k.take<EnsCluster>(C);
    e->active = k.take<int32_t>(N);
    e->flags = k.take<int32_t>(2);
    e->partial = k.take<double>((size_t)e->part_off_h[C]);
    e->crit = k.take<double>(2 * N);
    e->ek = k.take<double>(2 * C);
    e->ep = base ? e->ek + C : nullptr;
    return k.off;
}

nb_status ens_flags(nb_ens *e) {
    int32_t f[2];
    EHIP_OK(e, hipMemcpyAsync(f, e->flags, sizeof f, hipMemcpyDeviceToHost, e->stream));
    EHIP_OK(e, hipStreamSynchronize(e->stream));
    if (f[0]) return fail(e, NB_ENONFINITE, "non-finite force or state on device");
    if (f[1]) return fail(e, NB_EDTMIN, "time step below 2^-%d requested (clamped)", e->lmax);
    return NB_OK;
}

// nb_ens_run with independent lanes: each lane replays its own graph of global steps on its own
// stream, and the host checks a lane's clusters as soon as that lane's replay and the copy of
// the cluster records behind it have finished, then relaunches it, so no lane waits for another.
// The lanes start after the work already queued on the context's stream, which in turn waits
// for all of them before any later call.
nb_status ens_run_lanes(nb_ens *e, double eta, int64_t t_end, int32_t spl, int64_t max_steps,
                        int32_t use_graph) {
    const int L = e->lanes;
    if (use_graph && (!e->lane_gexec[0] || e->g_eta != eta || e->g_tend != t_end ||
                      e->g_steps != spl)) {
        ens_drop_graph(e);
        for (int l = 0; l < L; ++l) {
            EHIP_OK(e, hipStreamBeginCapture(e->cap_stream, hipStreamCaptureModeThreadLocal));
            nb_status rs = NB_OK;
            for (int32_t i = 0; i < spl && rs == NB_OK; ++i)
                rs = ens_enqueue_step(e, eta, t_end, e->cap_stream, l);
            hipGraph_t g = nullptr;
            hipError_t ec = hipStreamEndCapture(e->cap_stream, &g);
            if (rs != NB_OK) { if (g) (void)hipGraphDestroy(g); return rs; }
            if (ec != hipSuccess) return fail(e, NB_EDEVICE, "graph capture failed: %s", hipGetErrorString(ec));
            e->lane_graph[l] = g;
            EHIP_OK(e, hipGraphInstantiate(&e->lane_gexec[l], g, nullptr, nullptr, 0));
        }
        e->g_eta = eta; e->g_tend = t_end; e->g_steps = spl;
    }
    EHIP_OK(e, hipEventRecord(e->lane_join, e->stream));
    for (int l = 0; l < L; ++l) EHIP_OK(e, hipStreamWaitEvent(e->lane_stream[l], e->lane_join, 0));
    int64_t done_steps[ENS_MAX_LANES] = {}, prev[ENS_MAX_LANES];
    bool finished[ENS_MAX_LANES] = {};
    for (int l = 0; l < L; ++l) prev[l] = -1;
    auto launch = [&](int l) -> nb_status {
        const hipStream_t s = e->lane_stream[l];
        if (use_graph) {
            EHIP_OK(e, hipGraphLaunch(e->lane_gexec[l], s));
        } else {
            for (int32_t i = 0; i < spl; ++i) {
                const nb_status r = ens_enqueue_step(e, eta, t_end, s, l);
                if (r != NB_OK) return r;
            }
        }
        done_steps[l] += spl;
        EHIP_OK(e, hipMemcpyAsync(e->lane_host[l], e->cl, e->C * sizeof(EnsCluster),
                                  hipMemcpyDeviceToHost, s));
        EHIP_OK(e, hipEventRecord(e->lane_event[l], s));
        return NB_OK;
    };
    nb_status err = NB_OK;
    for (int l = 0; l < L && err == NB_OK; ++l) err = launch(l);
    int left = L;
    while (err == NB_OK && left > 0) {
        for (int l = 0; l < L && err == NB_OK; ++l) {
            if (finished[l]) continue;
            const hipError_t q = hipEventQuery(e->lane_event[l]);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) {
                err = fail(e, NB_EDEVICE, "lane %d: %s", l, hipGetErrorString(q));
                break;
            }
            bool all = true;
            int64_t total = 0;
            for (int32_t k = e->lane_start_h[l]; k < e->lane_start_h[l + 1]; ++k) {
                const EnsCluster &x = e->lane_host[l][e->order_h[k]];
                all = all && x.done;
                total += x.n_steps;
            }
            if (all || (max_steps > 0 && done_steps[l] >= max_steps)) {
                finished[l] = true;
                --left;
                continue;
            }
            // every global step advances every unfinished cluster by at least one block step
            if (total == prev[l]) {
                err = fail(e, NB_ESTATE, "ensemble lane %d made no progress over %d global steps", l, spl);
                break;
            }
            prev[l] = total;
            err = launch(l);
        }
    }
    for (int l = 0; l < L; ++l) {  // later work on the context's stream follows every lane
        (void)hipEventRecord(e->lane_event[l], e->lane_stream[l]);
        (void)hipStreamWaitEvent(e->stream, e->lane_event[l], 0);
    }
    if (err != NB_OK) {
        for (int l = 0; l < L; ++l) (void)hipStreamSynchronize(e->lane_stream[l]);
        return err;
    }
    return ens_flags(e);
}

}  // namespace

extern "C" {

const char *nb_ens_last_error(const nb_ens *e) { return e ? e->err.c_str() : "null ensemble"; }

nb_status nb_ens_create(nb_ens **out, int32_t n_clusters, const int32_t *offsets,
                        const double *eps, int32_t lmin, int32_t lmax, int32_t precision) {
    if (!out) return NB_EINVAL;
    *out = nullptr;
    if (!ens_args_ok(n_clusters, offsets, precision) || !eps || lmin < 0 || lmax < lmin ||
        lmax > 52)
        return NB_EINVAL;
    for (int32_t c = 0; c < n_clusters; ++c)
        if (!(eps[c] > 0.0) || !std::isfinite(eps[c])) return NB_EINVAL;
    nb_ens *e = new nb_ens();
    e->lmin = lmin; e->lmax = lmax;
    if (hipGetDevice(&e->device) != hipSuccess) { delete e; return NB_EDEVICE; }
    e->num_cu = device_cus(e->device);
    ens_plan(e, n_clusters, offsets, precision);
    e->eps2_h.resize(n_clusters);
    for (int32_t c = 0; c < n_clusters; ++c) e->eps2_h[c] = eps[c] * eps[c];
    e->scratch_need = ens_layout(e, nullptr);
    if (hipStreamCreateWithFlags(&e->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        delete e;
        return NB_EDEVICE;
    }
    *out = e;
    return NB_OK;
}

size_t nb_ens_scratch_bytes(int32_t n_clusters, const int32_t *offsets, int32_t precision) {
    if (!ens_args_ok(n_clusters, offsets, precision)) return 0;
    nb_ens e;
    ens_plan(&e, n_clusters, offsets, precision);
    return ens_layout(&e, nullptr);
}

nb_status nb_ens_bind_scratch(nb_ens *e, void *scratch, size_t bytes) {
    if (!e) return NB_EINVAL;
    if (!scratch) return fail(e, NB_EINVAL, "nb_ens_bind_scratch: workspace pointer required");
    if ((uintptr_t)scratch % 256 != 0)
        return fail(e, NB_EINVAL, "nb_ens_bind_scratch: workspace must be 256-byte aligned");
    if (bytes < e->scratch_need)
        return fail(e, NB_EINVAL, "nb_ens_bind_scratch: %zu bytes given, %zu needed", bytes,
                    e->scratch_need);
    EHIP_OK(e, hipSetDevice(e->device));
    EHIP_OK(e, hipStreamSynchronize(e->stream));
    ens_drop_graph(e);
    ens_layout(e, (char *)scratch);
    const size_t C = (size_t)e->C;
    EHIP_OK(e, hipMemcpyAsync(e->off, e->off_h.data(), (C + 1) * sizeof(int32_t), hipMemcpyHostToDevice, e->stream));
    EHIP_OK(e, hipMemcpyAsync(e->prow, e->prow_h.data(), C * sizeof(int32_t), hipMemcpyHostToDevice, e->stream));
    EHIP_OK(e, hipMemcpyAsync(e->order, e->order_h.data(), C * sizeof(int32_t), hipMemcpyHostToDevice, e->stream));
    EHIP_OK(e, hipMemcpyAsync(e->part_off, e->part_off_h.data(), (C + 1) * sizeof(int64_t), hipMemcpyHostToDevice, e->stream));
    EHIP_OK(e, hipMemcpyAsync(e->eps2, e->eps2_h.data(), C * sizeof(double), hipMemcpyHostToDevice, e->stream));
    EHIP_OK(e, hipMemcpyAsync(e->K, e->K_h.data(), C * sizeof(int32_t), hipMemcpyHostToDevice, e->stream));
    EHIP_OK(e, hipMemcpyAsync(e->tpi, e->tpi_h.data(), C * sizeof(int32_t), hipMemcpyHostToDevice, e->stream));
    ens_clear<<<std::max<int32_t>(1, (int32_t)((C + WG - 1) / WG)), WG, 0, e->stream>>>(e->cl, e->C, e->flags);
    ELAUNCH_OK(e);
    EHIP_OK(e, hipStreamSynchronize(e->stream));
    e->scratch_ok = true;
    e->initialised = false;
    return NB_OK;
}

nb_status nb_ens_destroy(nb_ens *e) {
    if (!e) return NB_OK;
    (void)hipSetDevice(e->device);
    (void)hipDeviceSynchronize();
    ens_drop_graph(e);
    if (e->cap_stream) (void)hipStreamDestroy(e->cap_stream);
    for (int l = 0; l < ENS_MAX_LANES; ++l) {
        if (e->lane_stream[l]) (void)hipStreamDestroy(e->lane_stream[l]);
        if (e->lane_event[l]) (void)hipEventDestroy(e->lane_event[l]);
        if (e->lane_host[l]) (void)hipHostFree(e->lane_host[l]);
    }
    if (e->lane_join) (void)hipEventDestroy(e->lane_join);
    delete e;
    return NB_OK;
}

nb_status nb_ens_set_stream(nb_ens *e, void *stream) {
    if (!e) return NB_EINVAL;
    e->stream = (hipStream_t)stream;
    return NB_OK;
}

nb_status nb_ens_bind(nb_ens *e, const nb_state *s) {
    if (!e || !s) return NB_EINVAL;
    if (!s->x || !s->v || !s->a || !s->k || !s->m || !s->pot || !s->tick || !s->level)
        return fail(e, NB_EINVAL, "nb_ens_bind: every state array is required");
    e->st = *s;
    e->bound = true;
    e->initialised = false;
    ens_drop_graph(e);
    return NB_OK;
}

nb_status nb_ens_set_layout(nb_ens *e, const int32_t *tiles_per_item, int32_t ipl, int32_t unroll) {
    if (!e) return NB_EINVAL;
    if (ipl != 1 || (unroll != 1 && unroll != 2))
        return fail(e, NB_EINVAL, "layout ipl=%d unroll=%d not available", ipl, unroll);
    if (tiles_per_item)
        for (int32_t c = 0; c < e->C; ++c)
            if (tiles_per_item[c] < 1) return fail(e, NB_EINVAL, "tiles per item must be >= 1");
    EHIP_OK(e, hipSetDevice(e->device));
    EHIP_OK(e, hipStreamSynchronize(e->stream));
    if (tiles_per_item) e->tpi_h.assign(tiles_per_item, tiles_per_item + e->C);
    e->unroll = unroll;
    ens_derive(e);
    ens_drop_graph(e);
    return ens_upload_tables(e);
}

nb_status nb_ens_set_split(nb_ens *e, int32_t smin) {
    if (!e) return NB_EINVAL;
    if (smin < 1 || smin > 64 || (smin & (smin - 1)) != 0)
        return fail(e, NB_EINVAL, "nb_ens_set_split: smin must be a power of two in [1, 64]");
    EHIP_OK(e, hipSetDevice(e->device));
    EHIP_OK(e, hipStreamSynchronize(e->stream));
    e->smin = smin;
    ens_derive(e);
    ens_drop_graph(e);
    return NB_OK;
}

nb_status nb_ens_set_lanes(nb_ens *e, int32_t lanes, const int32_t *lane_of) {
    if (!e) return NB_EINVAL;
    if (lanes < 1 || lanes > ENS_MAX_LANES)
        return fail(e, NB_EINVAL, "nb_ens_set_lanes: lanes must lie in [1, %d]", ENS_MAX_LANES);
    if (lanes > 1 && !lane_of) return fail(e, NB_EINVAL, "nb_ens_set_lanes: lane_of required");
    std::vector<int32_t> count(lanes, 0);
    for (int32_t c = 0; c < e->C; ++c) {
        const int32_t l = lanes > 1 ? lane_of[c] : 0;
        if (l < 0 || l >= lanes) return fail(e, NB_EINVAL, "nb_ens_set_lanes: cluster %d has lane %d", c, l);
        ++count[l];
    }
    for (int32_t l = 0; l < lanes; ++l)
        if (count[l] == 0) return fail(e, NB_EINVAL, "nb_ens_set_lanes: lane %d has no cluster", l);
    EHIP_OK(e, hipSetDevice(e->device));
    EHIP_OK(e, hipStreamSynchronize(e->stream));
    for (int32_t l = 0; l < lanes && lanes > 1; ++l) {  // streams at the default priority
        if (!e->lane_stream[l]) EHIP_OK(e, hipStreamCreateWithFlags(&e->lane_stream[l], hipStreamNonBlocking));
        if (!e->lane_event[l]) EHIP_OK(e, hipEventCreateWithFlags(&e->lane_event[l], hipEventDisableTiming));
        if (!e->lane_host[l])
            EHIP_OK(e, hipHostMalloc((void **)&e->lane_host[l], (size_t)e->C * sizeof(EnsCluster), hipHostMallocDefault));
    }
    if (lanes > 1 && !e->lane_join) EHIP_OK(e, hipEventCreateWithFlags(&e->lane_join, hipEventDisableTiming));
    // lane-major order table, each lane's clusters by decreasing size
    std::vector<int32_t> order, start(lanes + 1, 0);
    for (int32_t l = 0; l < lanes; ++l) {
        start[l] = (int32_t)order.size();
        for (int32_t c : e->size_order_h)
            if (lanes == 1 || lane_of[c] == l) order.push_back(c);
    }
    start[lanes] = e->C;
    e->order_h = order;
    e->lane_start_h = start;
    e->lanes = lanes;
    ens_drop_graph(e);
    if (e->scratch_ok) {
        EHIP_OK(e, hipMemcpyAsync(e->order, e->order_h.data(), e->C * sizeof(int32_t), hipMemcpyHostToDevice, e->stream));
        EHIP_OK(e, hipStreamSynchronize(e->stream));
    }
    return NB_OK;
}

nb_status nb_ens_set_local(nb_ens *e, int64_t local_limit, int32_t local_steps,
                           int64_t local_work) {
    if (!e) return NB_EINVAL;
    if (local_limit < 0 || local_steps < 0 || local_work < 0)
        return fail(e, NB_EINVAL, "local-step limits must be >= 0");
    EHIP_OK(e, hipSetDevice(e->device));
    EHIP_OK(e, hipStreamSynchronize(e->stream));
    e->local_limit = local_limit;
    e->local_steps = local_steps;
    e->local_work = local_work;
    ens_drop_graph(e);
    return NB_OK;
}

nb_status nb_ens_init(nb_ens *e, double eta) {
    if (!e) return NB_EINVAL;
    if (!e->scratch_ok) return fail(e, NB_ESTATE, "no workspace bound (call nb_ens_bind_scratch)");
    if (!e->bound) return fail(e, NB_ESTATE, "state not bound");
    if (!(eta > 0.0) || !std::isfinite(eta)) return fail(e, NB_EINVAL, "eta must be > 0");
    EHIP_OK(e, hipSetDevice(e->device));
    zero_words<<<1, WG, 0, e->stream>>>(nullptr, 0, e->flags, 2);
    ELAUNCH_OK(e);
    nb_status r;
    if ((r = ens_enqueue_local(e, eta, 0, INT64_MAX, e->stream, false)) != NB_OK) return r;
    if ((r = ens_enqueue_force(e, INT64_MAX, e->stream, false)) != NB_OK) return r;
    if ((r = ens_enqueue_local(e, eta, 1, INT64_MAX, e->stream, false)) != NB_OK) return r;
    e->initialised = true;
    return NB_OK;
}

nb_status nb_ens_run(nb_ens *e, double eta, int64_t t_end, int32_t steps_per_launch,
                     int64_t max_steps, int32_t use_graph) {
    if (!e) return NB_EINVAL;
    if (!e->initialised) return fail(e, NB_ESTATE, "nb_ens_run before nb_ens_init");
    if (!(eta > 0.0) || steps_per_launch < 1) return fail(e, NB_EINVAL, "bad arguments");
    EHIP_OK(e, hipSetDevice(e->device));
    if (e->lanes > 1) return ens_run_lanes(e, eta, t_end, steps_per_launch, max_steps, use_graph);
    if (use_graph && (!e->gexec || e->g_eta != eta || e->g_tend != t_end ||
                      e->g_steps != steps_per_launch)) {
        ens_drop_graph(e);
        EHIP_OK(e, hipStreamBeginCapture(e->cap_stream, hipStreamCaptureModeThreadLocal));
        nb_status rs = NB_OK;
        for (int32_t i = 0; i < steps_per_launch && rs == NB_OK; ++i)
            rs = ens_enqueue_step(e, eta, t_end, e->cap_stream);
        hipGraph_t g = nullptr;
        hipError_t ec = hipStreamEndCapture(e->cap_stream, &g);
        if (rs != NB_OK) { if (g) (void)hipGraphDestroy(g); return rs; }
        if (ec != hipSuccess) return fail(e, NB_EDEVICE, "graph capture failed: %s", hipGetErrorString(ec));
        e->graph = g;
        EHIP_OK(e, hipGraphInstantiate(&e->gexec, e->graph, nullptr, nullptr, 0));
        e->g_eta = eta; e->g_tend = t_end; e->g_steps = steps_per_launch;
    }
    std::vector<EnsCluster> h(e->C);
    int64_t done_steps = 0, prev_total = -1;
    for (;;) {
        if (use_graph) {
            EHIP_OK(e, hipGraphLaunch(e->gexec, e->stream));
        } else {
            for (int32_t i = 0; i < steps_per_launch; ++i) {
                nb_status r = ens_enqueue_step(e, eta, t_end, e->stream);
                if (r != NB_OK) return r;
            }
        }
        done_steps += steps_per_launch;
        EHIP_OK(e, hipMemcpyAsync(h.data(), e->cl, e->C * sizeof(EnsCluster), hipMemcpyDeviceToHost, e->stream));
        EHIP_OK(e, hipStreamSynchronize(e->stream));
        bool all = true;
        int64_t total = 0;
        for (const auto &x : h) {
            all = all && x.done;
            total += x.n_steps;
        }
        if (all || (max_steps > 0 && done_steps >= max_steps)) break;
        // every global step advances every unfinished cluster by at least one block step
        if (total == prev_total)
            return fail(e, NB_ESTATE, "ensemble made no progress over %d global steps", steps_per_launch);
        prev_total = total;
    }
    return ens_flags(e);
}

nb_status nb_ens_control(nb_ens *e, nb_control *out) {
    if (!e || !out) return NB_EINVAL;
    if (!e->scratch_ok) return fail(e, NB_ESTATE, "no workspace bound (call nb_ens_bind_scratch)");
    EHIP_OK(e, hipSetDevice(e->device));
    std::vector<EnsCluster> h(e->C);
    EHIP_OK(e, hipMemcpyAsync(h.data(), e->cl, e->C * sizeof(EnsCluster), hipMemcpyDeviceToHost, e->stream));
    EHIP_OK(e, hipStreamSynchronize(e->stream));
    for (int32_t c = 0; c < e->C; ++c) {
        out[c].t_cur = h[c].t_cur; out[c].t_next = h[c].t_next; out[c].t_end = e->g_tend;
        out[c].n_steps = h[c].n_steps; out[c].n_active_sum = h[c].n_active_sum;
        out[c].n_act = h[c].n_act; out[c].flags = h[c].done;
    }
    return ens_flags(e);
}

nb_status nb_ens_energy(nb_ens *e, double *ekin, double *epot) {
    if (!e || !ekin || !epot) return NB_EINVAL;
    if (!e->initialised) return fail(e, NB_ESTATE, "nb_ens_energy before nb_ens_init");
    EHIP_OK(e, hipSetDevice(e->device));
    ens_energy<<<e->C, WG, 0, e->stream>>>(ens_view(e, INT64_MAX), ens_state(e), e->ek, e->ep);
    ELAUNCH_OK(e);
    EHIP_OK(e, hipMemcpyAsync(ekin, e->ek, e->C * sizeof(double), hipMemcpyDeviceToHost, e->stream));
    EHIP_OK(e, hipMemcpyAsync(epot, e->ep, e->C * sizeof(double), hipMemcpyDeviceToHost, e->stream));
    EHIP_OK(e, hipStreamSynchronize(e->stream));
    return ens_flags(e);
}

}  // extern "C"
