// ensemble.hpp -- gfx950 device code for many independent clusters integrated together.
//
// Every cluster runs its own Sec. 2 block-step scheme (own times, levels and blocks).  One
// global step advances every unfinished cluster by one of its own block steps, in two kernels:
//   ens_force  all workgroups take work items (cluster, i-block, j-range); each workgroup
//              first forms the prefix over clusters of their item counts itself.  An item is an
//              i-block of the cluster's block against a range of whole j-tiles of the same
//              cluster; i- and j-particles are predicted to the cluster's block time as they
//              are loaded (Sec. 2 predictor, FP64); small blocks share each i among several
//              lanes (wave-shuffle reduction); partial sums go to the cluster's partial planes
//   ens_local  one workgroup of 1024 per cluster (largest clusters first): fixed-order sum of
//              the partials, the
//              corrector and the new step of each block particle (Eq. timestep), then the
//              cluster's next block (smallest t_i + dt_i)
// No workgroup ever waits for another: the cluster-local work needs only its own workgroup's
// barriers, and the phases are separate kernels.
#pragma once

#include "kernels.hpp"

namespace nbody {

struct EnsCluster {  // device-resident per-cluster record
    int64_t t_cur, t_next, n_steps, n_active_sum;
    int32_t n_act, n_pending, done, pad;
};

struct EnsView {
    int32_t C;                  // number of clusters
    const int32_t *off;         // C + 1 particle offsets
    const int32_t *K;           // j-ranges per i-block of each cluster
    const int32_t *tpi;         // whole tiles per j-range
    const int32_t *order;       // clusters by decreasing size: ens_local's workgroup order
    const int64_t *part_off;    // start of each cluster's partial planes
    const int32_t *prow;        // rows of one partial plane of each cluster
    const double *eps2;         // softening^2 of each cluster (> 0)
    EnsCluster *cl;
    int32_t *active;            // global indices, cluster c's block at active[off[c]...]
    double *partial;
    double *crit;
    int32_t *flags;             // [0]: non-finite seen, [1]: step clamped at 2^-lmax
    int32_t lmin, lmax;
    double tick_len;
    int64_t t_end;
    // Blocks advanced by the cluster's own workgroup (ens_local_block): at most local_limit
    // interactions (n_act * N_c; 0: none, every block goes through ens_force), and per launch
    // at most local_steps such block steps and local_work interactions per cluster.
    int64_t local_limit;
    int32_t local_steps;
    int64_t local_work;
    int32_t smin;               // fewest lanes per block particle in a force item (power of 2)
};

// Lanes per block particle of a cluster's force items: the lane split of its block, at least
// smin (smaller items, for balance across the GPU).
__host__ __device__ __forceinline__ int32_t ens_split(int32_t n_act, int32_t smin) {
    const int32_t S = lane_split(n_act, true);
    return S < smin ? smin : S;
}

constexpr int WGL = 1024;  // workgroup of the cluster-local kernel
constexpr int ENS_KMAX = 4; // j-ranges per cluster of the default force layout

// A cluster's selected block is forced by its own workgroup (and never by ens_force) when it
// holds at most WGL particles and at most `limit` interactions.
__host__ __device__ __forceinline__ bool ens_local_block(int32_t n_act, int32_t n_c, int64_t limit) {
    return n_act > 0 && n_act <= WGL && (int64_t)n_act * n_c <= limit;
}

// Fresh per-cluster records and flags (a fill kernel instead of a memset).
__global__ void __launch_bounds__(WG) ens_clear(EnsCluster *cl, int32_t C, int32_t *flags) {
    const int32_t c = blockIdx.x * WG + threadIdx.x;
    if (c < C) cl[c] = EnsCluster{0, 0, 0, 0, 0, 0, 0, 0};
    if (c < 2) flags[c] = 0;
}

// Ordered compaction of the particles of [lo, hi) that satisfy `pred` into out[base ...],
// by one workgroup; returns the count.
template <int BS, class Pred>
__device__ int32_t wg_compact(int32_t lo, int32_t hi, Pred pred, int32_t *out, int32_t *wsum) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int32_t base = 0;
    for (int32_t i0 = lo; i0 < hi; i0 += BS) {
        const int32_t i = i0 + threadIdx.x;
        const bool f = i < hi && pred(i);
        const uint64_t mask = __ballot(f);
        const int32_t below = __popcll(mask & ((1ull << lane) - 1ull));
        __syncthreads();
        if (lane == 0) wsum[wave] = __popcll(mask);
        __syncthreads();
        int32_t o = base;
        for (int w = 0; w < wave; ++w) o += wsum[w];
        if (f) out[o + below] = i;
        for (int w = 0; w < BS / 64; ++w) base += wsum[w];
    }
    return base;
}

template <int BS>
__device__ __forceinline__ int64_t block_min_i64(int64_t v, int64_t *red) {
    for (int off = 32; off > 0; off >>= 1) {
        const int64_t o = __shfl_xor(v, off, 64);
        v = o < v ? o : v;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    int64_t r = red[0];
    for (int w = 1; w < BS / 64; ++w) r = red[w] < r ? red[w] : r;
    return r;
}

constexpr int TN_CACHE = 4096;  // clusters up to this size keep t_i + dt_i in LDS for selection

// Predicted FP64 position and velocity of particle i at tick t (Sec. 2 predictor).
__device__ __forceinline__ void predicted(const StateRW &s, int32_t i, int64_t t, double xp[3],
                                          double vp[3]) {
    const double D = (double)(t - s.tick[i]) * s.tick_len;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int64_t ix = k * (int64_t)s.n + i;
        predict_one(D, s.x[ix], s.v[ix], s.a[ix], s.k[ix], xp[k], vp[k]);
    }
}

template <class M> __device__ __forceinline__ typename EpsOf<M>::T eps_as(double e2);
template <> __device__ __forceinline__ float eps_as<ModeF32>(double e2) { return (float)e2; }
template <> __device__ __forceinline__ ds eps_as<ModeDS>(double e2) { return ds_from_double(e2); }
template <> __device__ __forceinline__ double eps_as<ModeF64>(double e2) { return e2; }

// Next block among particles [lo, hi) by one workgroup of BS (Sec. 2: smallest t_i + dt_i, all
// particles attaining it, in ascending order) into out[0 ...]; every work-item gets the block
// size and time.  Returns false (n_act = 0) when the block lies beyond t_end.  Up to TN_CACHE
// particles keep t_i + dt_i in LDS for the compaction (tn_lds, TN_CACHE entries, may be NULL;
// the loads of several particles per work-item are issued together).
template <int BS>
__device__ bool block_select(const int64_t *tick, const int32_t *level, int32_t lo, int32_t hi,
                             int32_t lmax, int64_t t_end, int32_t *out, int64_t *tn_lds,
                             int64_t *red, int32_t *wsum, int32_t &n_act, int64_t &t_next) {
    const bool cached = tn_lds != nullptr && hi - lo <= TN_CACHE;
    int64_t m = INT64_MAX;
    if (cached) {
        int64_t tn[TN_CACHE / BS];
#pragma unroll
        for (int r = 0; r < TN_CACHE / BS; ++r) {
            const int32_t i = lo + threadIdx.x + r * BS;
            tn[r] = i < hi ? tick[i] + ((int64_t)1 << (lmax - level[i])) : INT64_MAX;
        }
#pragma unroll
        for (int r = 0; r < TN_CACHE / BS; ++r) {
            tn_lds[threadIdx.x + r * BS] = tn[r];
            m = tn[r] < m ? tn[r] : m;
        }
    } else {
        for (int32_t i = lo + threadIdx.x; i < hi; i += BS) {
            const int64_t tn = tick[i] + ((int64_t)1 << (lmax - level[i]));
            m = tn < m ? tn : m;
        }
    }
    const int64_t tn_min = block_min_i64<BS>(m, red);  // its barriers also publish tn_lds
    if (tn_min > t_end) {
        n_act = 0;
        return false;
    }
    n_act = cached
        ? wg_compact<BS>(lo, hi, [&](int32_t i) { return tn_lds[i - lo] == tn_min; }, out, wsum)
        : wg_compact<BS>(
              lo, hi,
              [&](int32_t i) { return tick[i] + ((int64_t)1 << (lmax - level[i])) == tn_min; },
              out, wsum);
    t_next = tn_min;
    __syncthreads();  // the block list is complete before any work-item reads it
    return true;
}

// Next block of cluster [lo, hi) into e.active[lo ...] and the cluster record (block_select);
// false when the cluster is done.
template <int BS>
__device__ bool ens_select(const EnsView &e, const StateRW &s, int32_t lo, int32_t hi,
                           EnsCluster *cl, int64_t *tn_lds, int64_t *red, int32_t *wsum,
                           int32_t &n_act, int64_t &t_next) {
    const bool more = block_select<BS>(s.tick, s.level, lo, hi, e.lmax, e.t_end, e.active + lo,
                                       tn_lds, red, wsum, n_act, t_next);
    if (threadIdx.x == 0) {
        if (more) {
            cl->t_next = t_next;
            cl->n_act = n_act;
        } else {
            cl->done = 1;
            cl->n_act = 0;
        }
    }
    return more;
}

// The 7 sums of block row q of cluster c over its K partial planes, in plane order (four
// planes' loads in flight).
__device__ __forceinline__ void ens_row_sums(const EnsView &e, int32_t c, int32_t q, double o[7]) {
    const int32_t K = e.K[c], P = e.prow[c];
    const int64_t stride = (int64_t)7 * P;
    const double *src = e.partial + e.part_off[c] + q;
#pragma unroll
    for (int k = 0; k < 7; ++k) o[k] = 0.0;
    int32_t j = 0;
    for (; j + 4 <= K; j += 4) {
        double v[4][7];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int k = 0; k < 7; ++k) v[r][k] = src[(j + r) * stride + (int64_t)k * P];
#pragma unroll
        for (int k = 0; k < 7; ++k) o[k] = (((o[k] + v[0][k]) + v[1][k]) + v[2][k]) + v[3][k];
    }
    for (; j < K; ++j) {
#pragma unroll
        for (int k = 0; k < 7; ++k) o[k] += src[j * stride + (int64_t)k * P];
    }
}

// Corrector of block particle i from its new sums (a, k in o[0..5], potential sum o[6]), new
// level from Eq. timestep.
__device__ __forceinline__ void ens_correct_one(const EnsView &e, const StateRW &s, int32_t i,
                                                int64_t t_next, const double o[7], double eta,
                                                bool &bad, bool &clamp) {
    const double a1[3] = {o[0], o[1], o[2]}, k1[3] = {o[3], o[4], o[5]};
    const double dt_old = (double)(t_next - s.tick[i]) * s.tick_len;
    double num = 0.0, den = 0.0;
    const bool ok = correct_particle(s, i, dt_old, a1, k1, -o[6], t_next, nullptr, &num, &den);
    bad = bad || !ok;
    const double dt = den > 0.0 ? __builtin_sqrt(eta * num / den) : __builtin_inf();
    bad = bad || __builtin_isnan(dt);
    clamp = clamp || dt < e.tick_len;
    s.level[i] = next_level(dt, s.level[i], t_next, e.lmin, e.lmax);
}

// The force of a block on particles [lo, hi) by one workgroup of BS (Sec. 2 Eq. Force with
// App. A softening, eps > 0): the block list `list` (global indices, n_act of them) against all
// particles of [lo, hi), predicted to t_next as they are staged in LDS, BS at a time.  S = BS /
// 2^ceil(log2 n_act) (at most 64, at least 1) adjacent lanes share a block particle and combine
// their sums by wave shuffles; longer lists take chunks of BS particles.  The 7 sums of row q
// (acc, jerk, and the potential sum taken positive) go to stage[k * ld + q].
template <class M, int BS>
__device__ void block_force_staged(const StateRW &s, int32_t lo, int32_t hi, const int32_t *list,
                                   int32_t n_act, int64_t t_next, typename EpsOf<M>::T eps2,
                                   typename M::Smem (&sm)[BS / TJ], double *stage, int64_t ld) {
    const int32_t n_c = hi - lo;
    int32_t p2 = 1;
    while (p2 < n_act && p2 < BS) p2 <<= 1;
    const int32_t Sl = BS / p2 > 64 ? 64 : BS / p2;
    const int32_t ib = BS / Sl;  // block particles per chunk
    const int32_t slice = (int32_t)threadIdx.x % Sl;
    for (int32_t q0 = 0; q0 < n_act; q0 += ib) {
        const int32_t q = q0 + (int32_t)threadIdx.x / Sl;
        const bool has = q < n_act;
        const int32_t g = has ? list[q] : lo;
        const int32_t own = has ? g - lo : -1;  // own slot among [lo, hi) (none on padding)
        double xp[3], vp[3];
        predicted(s, g, t_next, xp, vp);
        const typename M::I ii = M::make_i(xp, vp, s.m[g]);
        typename M::Sum S = M::sum_zero();
        for (int32_t t0 = 0; t0 < n_c; t0 += BS) {
            __syncthreads();
            const int32_t jl = t0 + (int32_t)threadIdx.x;
            typename M::Smem &st = sm[threadIdx.x / TJ];
            if (jl < n_c) {
                double xj[3], vj[3];
                predicted(s, lo + jl, t_next, xj, vj);
                M::put(st, threadIdx.x % TJ, xj, vj, s.m[lo + jl]);
            } else {  // padding: zero mass contributes nothing
                const double z[3] = {0.0, 0.0, 0.0};
                M::put(st, threadIdx.x % TJ, z, z, 0.0);
            }
            __syncthreads();
            const int32_t jn = n_c - t0 < BS ? n_c - t0 : BS;
            for (int b = 0; b * TJ < jn; ++b) {  // 256-slot sub-tiles, folded one at a time
                const int32_t cnt = jn - b * TJ < TJ ? jn - b * TJ : TJ;
                const int32_t rel = own - (t0 + b * TJ);
                typename M::Tile T = M::tile_zero();
                if (__ballot((uint32_t)rel < (uint32_t)cnt) != 0) {
#pragma unroll 2
                    for (int jj = slice; jj < cnt; jj += Sl)
                        M::template interact<true, true>(ii, sm[b], jj, eps2, T, jj == rel);
                } else {
#pragma unroll 2
                    for (int jj = slice; jj < cnt; jj += Sl)
                        M::template interact<true>(ii, sm[b], jj, eps2, T);
                }
                M::fold(S, T);
            }
        }
        for (int off = Sl >> 1; off > 0; off >>= 1) M::shfl_add(S, off);
        if (has && slice == 0) {
            const Out7 o = M::out(S);
#pragma unroll
            for (int k = 0; k < 7; ++k) stage[k * ld + q] = o.v[k];
        }
    }
    __syncthreads();  // the sums are complete, and every prediction read of the state is done
}

// One block step of a cluster by its own workgroup (the block is ens_local_block): the force
// (block_force_staged, sums staged in the cluster's first partial plane set), then the
// corrector and the new levels.
template <class M>
__device__ void ens_block_step_local(const EnsView &e, const StateRW &s, int32_t c, int32_t lo,
                                     int32_t hi, int32_t n_act, int64_t t_next, double eta,
                                     typename M::Smem (&sm)[WGL / TJ], bool &bad, bool &clamp) {
    double *stage = e.partial + e.part_off[c];
    const int64_t ld = e.prow[c];
    block_force_staged<M, WGL>(s, lo, hi, e.active + lo, n_act, t_next, eps_as<M>(e.eps2[c]), sm,
                               stage, ld);
    for (int32_t q = threadIdx.x; q < n_act; q += WGL) {
        double o[7];
#pragma unroll
        for (int k = 0; k < 7; ++k) o[k] = stage[k * ld + q];
        ens_correct_one(e, s, e.active[lo + q], t_next, o, eta, bad, clamp);
    }
    __syncthreads();  // the corrected times and levels precede the next selection
}

// One workgroup of WGL per cluster.
//   phase 0: start of run -- block = every particle, times 0, block time 0
//   phase 1: after the start-of-run force -- store a, k, pot and the initial levels
//            (Eq. initTimestep), then select the first block
//   phase 2: after a global force step -- correct the block ens_force computed (if it was not
//            a local block), give it new levels (Eq. timestep) and select the next block; then
//            advance the cluster by its own block steps while the selected block is a local
//            block, up to local_steps steps and local_work interactions
// The block ens_force computed: each thread takes whole block particles, the fixed-order sum of
// its K partial planes, the corrector and the new level, with the criterion in registers.
template <class M>
__global__ void __launch_bounds__(WGL) ens_local(EnsView e, StateRW s, double eta,
                                                 int32_t phase) {
    __shared__ int64_t red[WGL / 64];
    __shared__ int32_t wsum[WGL / 64];
    __shared__ int64_t tn_lds[TN_CACHE];
    __shared__ typename M::Smem sm[WGL / TJ];
    if ((int32_t)blockIdx.x >= e.C) return;
    // largest clusters first: the first wave of workgroups takes the longest ones and the
    // later, short ones fill in behind them
    const int32_t c = e.order[blockIdx.x];
    const int32_t lo = e.off[c], hi = e.off[c + 1];
    EnsCluster *cl = e.cl + c;
    if (phase == 0) {
        const int32_t na = wg_compact<WGL>(lo, hi, [](int32_t) { return true; }, e.active + lo, wsum);
        for (int32_t i = lo + threadIdx.x; i < hi; i += WGL) s.tick[i] = 0;
        if (threadIdx.x == 0) {
            cl->t_cur = 0; cl->t_next = 0; cl->n_steps = 0; cl->n_active_sum = 0;
            cl->n_act = na; cl->n_pending = 0; cl->done = 0;
        }
        return;
    }
    if (cl->done) return;  // n_act is already 0
    int32_t n_act = cl->n_act;
    int64_t t_next = cl->t_next;
    const int32_t n_c = hi - lo;
    bool bad = false, clamp = false;
    if (phase == 1 || !ens_local_block(n_act, n_c, e.local_limit)) {
        for (int32_t q = threadIdx.x; q < n_act; q += WGL) {
            double o[7];
            ens_row_sums(e, c, q, o);
            const int32_t i = e.active[lo + q];
            if (phase == 1) {
                double na = 0.0, nk = 0.0;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    s.a[k * (int64_t)s.n + i] = o[k];
                    s.k[k * (int64_t)s.n + i] = o[3 + k];
                    na = __builtin_fma(o[k], o[k], na);
                    nk = __builtin_fma(o[3 + k], o[3 + k], nk);
                }
                s.pot[i] = -o[6];
                na = __builtin_sqrt(na); nk = __builtin_sqrt(nk);
                const double dt = nk > 0.0 ? eta * na / nk : __builtin_inf();
                bad = bad || !__builtin_isfinite(na) || !__builtin_isfinite(nk);
                s.level[i] = level_from_dt(dt, e.lmin, e.lmax);
            } else {
                ens_correct_one(e, s, i, t_next, o, eta, bad, clamp);
            }
        }
        __syncthreads();
        if (phase == 2 && threadIdx.x == 0 && n_act > 0) {
            cl->t_cur = t_next;
            cl->n_steps += 1;
            cl->n_active_sum += n_act;
        }
        const bool more = ens_select<WGL>(e, s, lo, hi, cl, tn_lds, red, wsum, n_act, t_next);
        if (!more || phase == 1) {
            if (bad) e.flags[0] = 1;
            if (clamp) e.flags[1] = 1;
            return;
        }
    }
    // the cluster's own block steps while its blocks are small
    int64_t work = 0;
    for (int32_t it = 0; it < e.local_steps && work < e.local_work &&
                         ens_local_block(n_act, n_c, e.local_limit); ++it) {
        ens_block_step_local<M>(e, s, c, lo, hi, n_act, t_next, eta, sm, bad, clamp);
        work += (int64_t)n_act * n_c;
        if (threadIdx.x == 0) {
            cl->t_cur = t_next;
            cl->n_steps += 1;
            cl->n_active_sum += n_act;
        }
        if (!ens_select<WGL>(e, s, lo, hi, cl, tn_lds, red, wsum, n_act, t_next)) break;
    }
    if (bad) e.flags[0] = 1;
    if (clamp) e.flags[1] = 1;
}

// ------------------------------------------------------------------------------------------
// Block steps of one small particle set by one resident workgroup, its whole state in LDS.
// ------------------------------------------------------------------------------------------
constexpr int RES_MAX = 1024;  // particles whose FP64 state (116 B each) one workgroup keeps in LDS
constexpr int RES_NT = 2;      // j sub-tiles of TJ staged per pass
static_assert(RES_MAX <= WGL, "the resident selection takes one particle per work-item");

// Next block of a set of n <= WGL particles (one per work-item) by one workgroup of WGL: the
// smallest t_i + dt_i (Sec. 2) and every particle attaining it, in ascending order, into
// out[0 ...].  Three barriers: wave minima, then wave counts of the block, then the list.
// Returns false (n_act = 0) when the block lies beyond t_end; red and cnt are LDS scratch of
// WGL / 64 entries each, free again when this returns.
__device__ bool resident_select(const int64_t *tick, const int32_t *level, int32_t n,
                                int32_t lmax, int64_t t_end, int32_t *out, int64_t *red,
                                int32_t *cnt, int32_t &n_act, int64_t &t_next) {
    const int32_t i = threadIdx.x;
    const int lane = i & 63, wave = i >> 6;
    const int64_t tn = i < n ? tick[i] + ((int64_t)1 << (lmax - level[i])) : INT64_MAX;
    int64_t m = tn;
    for (int off = 32; off > 0; off >>= 1) {
        const int64_t o = __shfl_xor(m, off, 64);
        m = o < m ? o : m;
    }
    if (lane == 0) red[wave] = m;
    __syncthreads();
    int64_t t_min = red[0];
#pragma unroll
    for (int w = 1; w < WGL / 64; ++w) t_min = red[w] < t_min ? red[w] : t_min;
    if (t_min > t_end) {
        n_act = 0;
        return false;
    }
    const bool f = tn == t_min;
    const uint64_t mask = __ballot(f);
    if (lane == 0) cnt[wave] = __popcll(mask);
    __syncthreads();
    int32_t below = 0, total = 0;
#pragma unroll
    for (int w = 0; w < WGL / 64; ++w) {
        const int32_t c = cnt[w];
        below += w < wave ? c : 0;
        total += c;
    }
    if (f) out[below + __popcll(mask & ((1ull << lane) - 1ull))] = i;
    // equal on every work-item: kept in scalar registers
    n_act = __builtin_amdgcn_readfirstlane(total);
    t_next = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(t_min >> 32)) << 32) |
                       (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)t_min));
    __syncthreads();  // the list is complete, and red and cnt may be written again
    return true;
}

// The force of the block `list` (n_act <= n <= WGL particles, one pass: S lanes per block
// particle with S * 2^ceil(log2 n_act) <= WGL) against all n particles predicted to t_next as
// they are staged RES_NT sub-tiles at a time (Sec. 2 Eq. Force, App. A softening, j != i), then
// the corrector and the new level of each block particle by the lane that holds its sums.
// Waves whose slots are all past the block only stage.  The state is read only while staging
// and predicting the i-particles, so the correctors need no barrier before their writes.
template <class M>
__device__ void resident_force_correct(const StateRW &s, const int32_t *list, int32_t n_act,
                                       int64_t t_next, typename EpsOf<M>::T eps2,
                                       typename M::Smem (&sm)[RES_NT], double eta, int32_t lmin,
                                       int32_t lmax, bool &bad, bool &clamp) {
    const int32_t n = s.n;
    int32_t p2 = 1;
    while (p2 < n_act) p2 <<= 1;
    const int32_t Sl = WGL / p2 > 64 ? 64 : WGL / p2;
    const int32_t q = (int32_t)threadIdx.x / Sl, slice = (int32_t)threadIdx.x % Sl;
    const bool has = q < n_act;
    const bool busy = (int32_t)(threadIdx.x & ~63u) / Sl < n_act;  // wave-uniform
    const int32_t g = has ? list[q] : 0;
    const int32_t own = has ? g : -1;  // own slot (none on padding)
    double xp[3], vp[3];
    predicted(s, g, t_next, xp, vp);
    const typename M::I ii = M::make_i(xp, vp, s.m[g]);
    typename M::Sum S = M::sum_zero();
    for (int32_t t0 = 0; t0 < n; t0 += RES_NT * TJ) {
        __syncthreads();  // the previous pass's tiles are consumed
        if (threadIdx.x < RES_NT * TJ) {
            const int32_t jl = t0 + (int32_t)threadIdx.x;
            typename M::Smem &st = sm[threadIdx.x / TJ];
            if (jl < n) {
                double xj[3], vj[3];
                predicted(s, jl, t_next, xj, vj);
                M::put(st, threadIdx.x % TJ, xj, vj, s.m[jl]);
            } else {  // padding: zero mass contributes nothing
                const double z[3] = {0.0, 0.0, 0.0};
                M::put(st, threadIdx.x % TJ, z, z, 0.0);
            }
        }
        __syncthreads();
        if (!busy) continue;
        const int32_t jn = n - t0 < RES_NT * TJ ? n - t0 : RES_NT * TJ;
        for (int b = 0; b * TJ < jn; ++b) {  // 256-slot sub-tiles, folded one at a time
            const int32_t cnt = jn - b * TJ < TJ ? jn - b * TJ : TJ;
            const int32_t rel = own - (t0 + b * TJ);
            typename M::Tile T = M::tile_zero();
            if (__ballot((uint32_t)rel < (uint32_t)cnt) != 0) {
#pragma unroll 2
                for (int jj = slice; jj < cnt; jj += Sl)
                    M::template interact<true, true>(ii, sm[b], jj, eps2, T, jj == rel);
            } else {
#pragma unroll 2
                for (int jj = slice; jj < cnt; jj += Sl)
                    M::template interact<true>(ii, sm[b], jj, eps2, T);
            }
            M::fold(S, T);
        }
    }
    if (!busy) return;
    for (int off = Sl >> 1; off > 0; off >>= 1) M::shfl_add(S, off);
    if (!has || slice != 0) return;
    const Out7 o = M::out(S);
    const double a1[3] = {o.v[0], o.v[1], o.v[2]}, k1[3] = {o.v[3], o.v[4], o.v[5]};
    const double dt_old = (double)(t_next - s.tick[g]) * s.tick_len;
    double num = 0.0, den = 0.0;
    bad = bad || !correct_particle(s, g, dt_old, a1, k1, -o.v[6], t_next, nullptr, &num, &den);
    const double dt = den > 0.0 ? __builtin_sqrt(eta * num / den) : __builtin_inf();
    bad = bad || __builtin_isnan(dt);
    clamp = clamp || dt < s.tick_len;
    s.level[g] = next_level(dt, s.level[g], t_next, lmin, lmax);
}

// Block steps of one particle set of n <= RES_MAX by one resident workgroup, for sets so small
// that a block step is far shorter than a chain of kernel launches.  The FP64 state (x, v, a,
// k, m, tick, level) is loaded into LDS once per launch and written back at its end; each pass
// of the loop selects the next block up to the scheduler's t_end (resident_select, into an
// LDS list), forces and corrects it (resident_force_correct), repeated up to `steps` times or until
// no block lies at or before t_end.  Potentials go straight to the state's pot, the last block
// stepped to `active`.  The scheduler record is the context's (block time and size, step
// counters, latched flags).
template <class M>
__global__ void __launch_bounds__(WGL) run_resident(StateRW g, int32_t *active, DevControl *ctl,
                                                    double eps2, double eta, int32_t lmin,
                                                    int32_t lmax, int32_t steps) {
    __shared__ double lx[3 * RES_MAX], lv[3 * RES_MAX], la[3 * RES_MAX], lk[3 * RES_MAX];
    __shared__ double lm[RES_MAX];
    __shared__ int64_t ltick[RES_MAX];
    __shared__ int32_t llevel[RES_MAX], lact[RES_MAX];
    __shared__ int64_t red[WGL / 64];
    __shared__ int32_t wcnt[WGL / 64];
    __shared__ typename M::Smem sm[RES_NT];
    const int32_t n = g.n;
    if (n > RES_MAX || ctl->done) return;  // every work-item reads the same record
    const int64_t t_end = ctl->t_end;
    for (int32_t e = threadIdx.x; e < 3 * n; e += WGL) {
        lx[e] = g.x[e];
        lv[e] = g.v[e];
        la[e] = g.a[e];
        lk[e] = g.k[e];
    }
    for (int32_t i = threadIdx.x; i < n; i += WGL) {
        lm[i] = g.m[i];
        ltick[i] = g.tick[i];
        llevel[i] = g.level[i];
    }
    StateRW s = g;
    s.x = lx; s.v = lv; s.a = la; s.k = lk; s.m = lm; s.tick = ltick; s.level = llevel;
    __syncthreads();
    bool bad = false, clamp = false, done = false;
    int32_t n_last = 0, stepped = 0;  // size of the last block stepped; block steps taken
    int64_t t_last = 0, act_sum = 0;
    for (int32_t it = 0; it < steps; ++it) {
        int32_t n_act = 0;
        int64_t t_next = 0;
        if (!resident_select(s.tick, s.level, n, lmax, t_end, lact, red, wcnt, n_act, t_next)) {
            done = true;
            break;
        }
        resident_force_correct<M>(s, lact, n_act, t_next, eps_as<M>(eps2), sm, eta, lmin, lmax,
                                  bad, clamp);
        n_last = n_act;
        t_last = t_next;
        stepped += 1;
        act_sum += n_act;
        __syncthreads();  // corrected times and levels precede the next selection
    }
    // the scheduler record once per launch (every work-item holds the same counts)
    if (threadIdx.x == 0) {
        ctl->n_pending = 0;  // levels are current
        if (stepped > 0) {
            ctl->t_cur = t_last;
            ctl->t_next = t_last;
            ctl->n_steps += stepped;
            ctl->n_active_sum += act_sum;
        }
        ctl->n_act = done ? 0 : n_last;
        if (done) ctl->done = 1;
    }
    __syncthreads();
    for (int32_t e = threadIdx.x; e < 3 * n; e += WGL) {
        g.x[e] = lx[e];
        g.v[e] = lv[e];
        g.a[e] = la[e];
        g.k[e] = lk[e];
    }
    for (int32_t i = threadIdx.x; i < n; i += WGL) {
        g.tick[i] = ltick[i];
        g.level[i] = llevel[i];
    }
    for (int32_t q = threadIdx.x; q < n_last; q += WGL) active[q] = lact[q];  // the last block
    if (bad) ctl->flag_nonfinite = 1;
    if (clamp) ctl->flag_dtmin = 1;
}

// Exclusive prefix of the clusters' force work items (ens_item: i-blocks of WG / S block
// particles times K j-ranges) in the size order (largest cluster first, so the largest items
// go to the first wave of workgroups and the small ones fill in behind), start[0..C] indexed by
// place in that order, formed by one workgroup of BS in its LDS: each work-item takes a
// contiguous run of places, the runs' totals are scanned across the wave (shuffles) and across
// waves (wsum).
template <int BS>
__device__ void ens_item_prefix(const EnsView &e, int32_t *start, int32_t *wsum) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int32_t per = (e.C + BS - 1) / BS;
    const int32_t c0 = (int32_t)threadIdx.x * per;
    const int32_t c1 = c0 + per < e.C ? c0 + per : e.C;
    int32_t own = 0;
    for (int32_t k = c0; k < c1; ++k) {  // k: place in the size order, cluster e.order[k]
        const int32_t c = e.order[k];
        const int32_t na = e.cl[c].n_act;
        const int32_t ibc = WG / ens_split(na, e.smin);  // i-block of an item (ens_item), any BS
        const bool global = na > 0 && !ens_local_block(na, e.off[c + 1] - e.off[c], e.local_limit);
        const int32_t items = global ? ((na + ibc - 1) / ibc) * e.K[c] : 0;
        start[k] = items;
        own += items;
    }
    int32_t inc = own;  // inclusive scan over the wave
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t v = __shfl_up(inc, o, 64);
        if (lane >= o) inc += v;
    }
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    int32_t run = inc - own;
    for (int w = 0; w < wave; ++w) run += wsum[w];
    for (int32_t k = c0; k < c1; ++k) {
        const int32_t items = start[k];
        start[k] = run;
        run += items;
    }
    if (threadIdx.x == BS - 1) start[e.C] = run;
    __syncthreads();
}

// Place (in the size order) of the cluster of item w: the last k with start[k] <= w.
__device__ __forceinline__ int32_t ens_item_cluster(const int32_t *start, int32_t C, int32_t w) {
    int32_t lo = 0, hi = C - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (start[mid] <= w) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Force work item `local` of cluster c (its i-block of the block list against its range of
// whole j-tiles), partial sums to the cluster's planes.  Softened (eps > 0) interactions only;
// one i per work-item, S lanes per i when the cluster's block is small.
template <class M, int UNR>
__device__ void ens_item(const EnsView &e, const StateRW &st, int32_t c, int32_t local,
                         typename M::Smem &sm) {
    const int32_t K = e.K[c], tpi = e.tpi[c];
    const int32_t iblk = local / K, ks = local - (local / K) * K;
    const int32_t p0 = e.off[c], n_c = e.off[c + 1] - p0;
    const int32_t n_act = e.cl[c].n_act;
    const int64_t tb = e.cl[c].t_next;
    const int32_t Sl = ens_split(n_act, e.smin);
    const int32_t slice = (int32_t)threadIdx.x % Sl;
    const int32_t ntiles = (n_c + TJ - 1) / TJ;
    const auto eps2 = eps_as<M>(e.eps2[c]);
    const int32_t q = iblk * (WG / Sl) + (int32_t)threadIdx.x / Sl;
    const int32_t g = q < n_act ? e.active[p0 + q] : p0;
    const int32_t own = q < n_act ? g - p0 : -1;  // own slot in the cluster (none on padding)
    double xp[3], vp[3];
    predicted(st, g, tb, xp, vp);
    const typename M::I ii = M::make_i(xp, vp, st.m[g]);
    typename M::Sum S = M::sum_zero();
    const int32_t t0 = ks * tpi;
    const int32_t t1 = t0 + tpi < ntiles ? t0 + tpi : ntiles;
    for (int32_t t = t0; t < t1; ++t) {
        __syncthreads();
        const int32_t jl = t * TJ + (int32_t)threadIdx.x;
        if (jl < n_c) {
            double xj[3], vj[3];
            predicted(st, p0 + jl, tb, xj, vj);
            M::put(sm, threadIdx.x, xj, vj, st.m[p0 + jl]);
        } else {  // padding: zero mass contributes nothing
            const double z[3] = {0.0, 0.0, 0.0};
            M::put(sm, threadIdx.x, z, z, 0.0);
        }
        __syncthreads();
        typename M::Tile T = M::tile_zero();
        const int32_t jn = n_c - t * TJ < TJ ? n_c - t * TJ : TJ;  // padding is skipped
        // a tile holding a lane's own particle takes the masked loop (wave-uniform branch)
        const int32_t rel = own - t * TJ;
        if (__ballot((uint32_t)rel < (uint32_t)jn) != 0) {
#pragma unroll UNR
            for (int jj = slice; jj < jn; jj += Sl)
                M::template interact<true, true>(ii, sm, jj, eps2, T, jj == rel);
        } else {
#pragma unroll UNR
            for (int jj = slice; jj < jn; jj += Sl) M::template interact<true>(ii, sm, jj, eps2, T);
        }
        M::fold(S, T);
    }
    for (int off = Sl >> 1; off > 0; off >>= 1) M::shfl_add(S, off);
    if (slice == 0 && q < n_act) {
        const Out7 o = M::out(S);
        const int32_t P = e.prow[c];
        double *base = e.partial + e.part_off[c] + (int64_t)ks * 7 * P + q;
#pragma unroll
        for (int k = 0; k < 7; ++k) base[(int64_t)k * P] = o.v[k];
    }
}

// The force items of every cluster's block (those that are not local blocks).
// Dynamic LDS: the C + 1 item starts, formed once per workgroup.
template <class M, int UNR>
__global__ void __launch_bounds__(WG) ens_force(EnsView e, StateRW st) {
    __shared__ typename M::Smem sm;
    __shared__ int32_t wsum[WG / 64];
    extern __shared__ int32_t start[];
    ens_item_prefix<WG>(e, start, wsum);
    const int32_t total = start[e.C];
    for (int32_t w = blockIdx.x; w < total; w += gridDim.x) {
        const int32_t k = ens_item_cluster(start, e.C, w);
        ens_item<M, UNR>(e, st, e.order[k], w - start[k], sm);
    }
}

// Energy of every cluster at its current time (FP64): one workgroup per cluster, pair sums
// with Neumaier compensation; cluster particles predicted to the cluster's t_cur.
__global__ void __launch_bounds__(WG) ens_energy(EnsView e, StateRW s, double *ekin,
                                                 double *epot) {
    __shared__ double sx[TJ], sy[TJ], sz[TJ], smm[TJ];
    __shared__ double rk[WG], rp[WG];
    const int32_t c = blockIdx.x;
    if (c >= e.C) return;
    const int32_t p0 = e.off[c], n_c = e.off[c + 1] - p0;
    const int64_t t = e.cl[c].t_cur;
    const double eps2 = e.eps2[c];
    double kin = 0.0, kc = 0.0, pot = 0.0, pc = 0.0;
    for (int32_t i0 = 0; i0 < n_c; i0 += WG) {
        const int32_t il = i0 + threadIdx.x;
        const int32_t i = p0 + (il < n_c ? il : 0);
        const double D = (double)(t - s.tick[i]) * s.tick_len;
        double xi[3], vi[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int64_t ix = k * (int64_t)s.n + i;
            predict_one(D, s.x[ix], s.v[ix], s.a[ix], s.k[ix], xi[k], vi[k]);
        }
        double w = 0.0, wc = 0.0;
        for (int32_t j0 = 0; j0 < n_c; j0 += TJ) {
            __syncthreads();
            const int32_t jl = j0 + threadIdx.x;
            if (jl < n_c) {
                const int32_t j = p0 + jl;
                const double Dj = (double)(t - s.tick[j]) * s.tick_len;
                double xj[3], vj[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const int64_t ix = k * (int64_t)s.n + j;
                    predict_one(Dj, s.x[ix], s.v[ix], s.a[ix], s.k[ix], xj[k], vj[k]);
                }
                sx[threadIdx.x] = xj[0]; sy[threadIdx.x] = xj[1]; sz[threadIdx.x] = xj[2];
                smm[threadIdx.x] = s.m[j];
            } else {
                sx[threadIdx.x] = 0.0; sy[threadIdx.x] = 0.0; sz[threadIdx.x] = 0.0;
                smm[threadIdx.x] = 0.0;
            }
            __syncthreads();
            double ts = 0.0;
            const int32_t cnt = n_c - j0 < TJ ? n_c - j0 : TJ;
            for (int jj = 0; jj < cnt; ++jj) {
                const double dx = sx[jj] - xi[0], dy = sy[jj] - xi[1], dz = sz[jj] - xi[2];
                const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, __builtin_fma(dx, dx, eps2)));
                ts += (j0 + jj == il) ? 0.0 : smm[jj] * rsqrt_f64(r2);
            }
            const double y = w + ts;
            wc += __builtin_fabs(w) >= __builtin_fabs(ts) ? (w - y) + ts : (ts - y) + w;
            w = y;
        }
        if (il < n_c) {
            const double mi = s.m[i];
            const double pe = mi * (w + wc);
            const double ke = 0.5 * mi * __builtin_fma(vi[2], vi[2], __builtin_fma(vi[1], vi[1], vi[0] * vi[0]));
            double y = pot + pe;
            pc += __builtin_fabs(pot) >= __builtin_fabs(pe) ? (pot - y) + pe : (pe - y) + pot;
            pot = y;
            y = kin + ke;
            kc += __builtin_fabs(kin) >= __builtin_fabs(ke) ? (kin - y) + ke : (ke - y) + kin;
            kin = y;
        }
    }
    rk[threadIdx.x] = kin + kc;
    rp[threadIdx.x] = pot + pc;
    __syncthreads();
    for (int o = WG / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            rk[threadIdx.x] += rk[threadIdx.x + o];
            rp[threadIdx.x] += rp[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        ekin[c] = rk[0];
        epot[c] = -0.5 * rp[0];
    }
}

}  // namespace nbody
