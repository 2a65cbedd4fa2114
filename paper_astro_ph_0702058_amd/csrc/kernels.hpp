// kernels.hpp -- gfx950 device code of libnbody.
//
// Hermite block-step direct N-body integration (Portegies Zwart, Belleman & Geldof 2007):
//   predict       Sec. 2 predictor, FP64, all particles -> the j-particle stream
//   force_kernel  Sec. 2 Eq. Force with App. A softening: acceleration, jerk, potential of a
//                 list of i-particles against all predicted j-particles (FP32 / DS / FP64)
//   force_reduce  fixed-order sum of the j-split partial sums
//   correct       Sec. 2 corrector, FP64, on the block
//   sched_*       Sec. 2 block selection and Eq. timestep, integer time in ticks
//   energy_*      Sec. 4.2 energy diagnostic, FP64
// Wave64 throughout; workgroups of 256 work-items (4 waves).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ds_arith.hpp"

namespace nbody {

constexpr int WG = 256;      // work-items per workgroup
constexpr int TJ = 256;      // j-particles per tile (LDS tile of the lane split; fold interval)

// Device-side scheduler record.  The first 48 bytes mirror nb_control of the C ABI.
struct DevControl {
    int64_t t_cur;
    int64_t t_next;
    int64_t t_end;
    int64_t n_steps;
    int64_t n_active_sum;
    int32_t n_act;
    int32_t flags;          // unused on device; flags live in the words below
    // internal
    int64_t t_cand;         // smallest t_i + dt_i found by the last selection
    int32_t n_pending;      // particles corrected but not yet given a new level
    int32_t done;           // the last selection found no block at or before t_end
    int32_t flag_nonfinite; // latched: a force or corrected state was not finite
    int32_t flag_dtmin;     // latched: the criterion asked for a step below 2^-lmax
    // fused block step
    int32_t flag_sched;     // latched: a particle's next time preceded the block time
    int32_t pad_;
    int32_t hist[64];       // particles per level
    // fused selection: block members appended so far (low word) and chunks finished (high
    // word); zero between steps
    uint64_t sel;
};

// ------------------------------------------------------------------------------------------
// Work decomposition of one force call, computed identically on host and device from the
// number of i-particles: i-blocks of WG*IPL particles times K contiguous j-ranges (whole
// tiles).  K > 1 only when the i-blocks alone cannot fill `target` work items.
// ------------------------------------------------------------------------------------------
struct ForcePlan {
    int32_t n_i, n_iblk, ntiles, tps, K, items;
    int32_t S;   // lanes sharing one i-particle (1 unless the i-list is small)
    int32_t ib;  // i-particles per i-block
    int64_t P;   // padded i rows of one partial plane
};

// Lanes per i-particle for a list of n_i with one i per work-item: the whole workgroup is
// spread over the list, up to smax lanes (at most one wave) per i.
__host__ __device__ inline int32_t lane_split(int32_t n_i, bool allowed, int32_t smax = 64) {
    if (!allowed || n_i >= WG) return 1;
    int32_t p2 = 1;
    while (p2 < n_i) p2 <<= 1;
    const int32_t S = WG / p2;
    return S > smax ? smax : S;
}

// ib_max: WG * (i-particles per work-item).  Lists shorter than a workgroup take the lane
// split whatever the variant (one i per group of S lanes), so that a short block costs work in
// proportion to its length.
__host__ __device__ inline ForcePlan make_plan(int32_t n_i, int32_t n, int32_t ib_max,
                                               int32_t target, int32_t kmax, int32_t smax = 64) {
    ForcePlan p;
    p.n_i = n_i;
    p.S = lane_split(n_i, true, smax);
    const int32_t ib = p.S > 1 ? WG / p.S : ib_max;
    p.ib = ib;
    p.n_iblk = (n_i + ib - 1) / ib;
    p.ntiles = (n + TJ - 1) / TJ;
    int32_t K = p.n_iblk > 0 ? target / p.n_iblk : 1;
    if (K > kmax) K = kmax;
    if (K > p.ntiles) K = p.ntiles;
    if (K < 1) K = 1;
    p.tps = (p.ntiles + K - 1) / K;
    p.K = (p.ntiles + p.tps - 1) / p.tps;
    p.items = p.n_iblk * p.K;
    p.P = (int64_t)p.n_iblk * ib;
    return p;
}

struct ForceCommon {
    int32_t n;               // number of j-particles
    const int32_t *ilist;    // i-particle indices (NULL: identity)
    const int32_t *n_i_dev;  // device count (NULL: n_i_max)
    int32_t n_i_max;
    int32_t target;          // desired work items
    int32_t kmax;            // largest j-split
    double *acc, *jerk, *pot;
    int32_t ld;              // leading dimension of acc/jerk/pot
    double *partial;         // K > 1: [K][7][P]
    DevControl *ctl;         // latched flags (may be NULL)
    int32_t smax;            // largest lane split of the arithmetic mode
    int32_t scalar_min;      // fewest j-tiles per item read with scalar loads (float modes)
};

// Sum record written per i-particle: acc (3), jerk (3), accumulated m/r (1).
struct Out7 {
    double v[7];
};

// Wave-uniform reads of j-records: on the whole-block path every lane of a wave takes the same
// j at the same time, so the record is read once per wave through the scalar data cache into
// scalar registers, which the vector instructions take as operands (the j-stream is read-only
// while a force launch runs).
typedef float f4v __attribute__((ext_vector_type(4)));
__device__ __forceinline__ double uload(const double *p, int j) {
    return ((const __attribute__((address_space(4))) double *)p)[j];
}
__device__ __forceinline__ float4 uload(const float4 *p, int j) {
    const f4v q = ((const __attribute__((address_space(4))) f4v *)p)[j];
    return make_float4(q.x, q.y, q.z, q.w);
}

// ------------------------------------------------------------------------------------------
// FP32 interaction: separations from FP64 positions (one rounding), float arithmetic, tile
// sums in float folded into double sums once per tile.
// ------------------------------------------------------------------------------------------
struct ModeF32 {
    struct Args {
        const double *px, *py, *pz;
        const float4 *vm;  // vx, vy, vz, m
        float eps2;
    };
    struct I {
        double x, y, z;
        float vx, vy, vz, m;
    };
    struct Smem {
        double x[TJ], y[TJ], z[TJ];
        float4 vm[TJ];
    };
    struct Tile {
        float ax, ay, az, jx, jy, jz, p;
    };
    struct Sum {
        double ax, ay, az, jx, jy, jz, p;
    };

    __device__ static I load_i(const Args &a, int g) {
        const float4 q = a.vm[g];
        return I{a.px[g], a.py[g], a.pz[g], q.x, q.y, q.z, q.w};
    }
    __device__ static void stage(const Args &a, Smem &s, int t, int j, int n) {
        if (j < n) {
            s.x[t] = a.px[j]; s.y[t] = a.py[j]; s.z[t] = a.pz[j]; s.vm[t] = a.vm[j];
        } else {  // padding: zero mass contributes nothing
            s.x[t] = 0.0; s.y[t] = 0.0; s.z[t] = 0.0; s.vm[t] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
    }
    __device__ static Tile tile_zero() { return Tile{0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f}; }
    __device__ static Sum sum_zero() { return Sum{0., 0., 0., 0., 0., 0., 0.}; }
    // records built directly from FP64 predicted values (as the predictor would write them)
    __device__ static I make_i(const double xp[3], const double vp[3], double m) {
        return I{xp[0], xp[1], xp[2], (float)vp[0], (float)vp[1], (float)vp[2], (float)m};
    }
    __device__ static void put(Smem &s, int t, const double xp[3], const double vp[3], double m) {
        s.x[t] = xp[0]; s.y[t] = xp[1]; s.z[t] = xp[2];
        s.vm[t] = make_float4((float)vp[0], (float)vp[1], (float)vp[2], (float)m);
    }

    struct J {  // one j-record
        double x, y, z;
        float4 q;
    };
    __device__ static __forceinline__ J load_j(const Args &a, int j) {
        return J{uload(a.px, j), uload(a.py, j), uload(a.pz, j), uload(a.vm, j)};
    }
    template <bool SOFT, bool MASK = false>
    __device__ static __forceinline__ void interact(const I &i, const Smem &s, int jj, float eps2,
                                                    Tile &T, bool self = false) {
        pair<SOFT, MASK>(i, J{s.x[jj], s.y[jj], s.z[jj], s.vm[jj]}, eps2, T, self);
    }
    // MASK: the pair may be the i-particle's own slot (self), which then adds nothing
    template <bool SOFT, bool MASK = false>
    __device__ static __forceinline__ void pair(const I &i, const J &j, float eps2, Tile &T,
                                                bool self = false) {
        const float dx = (float)(j.x - i.x);
        const float dy = (float)(j.y - i.y);
        const float dz = (float)(j.z - i.z);
        const float4 q = j.q;
        const float ux = q.x - i.vx;
        const float uy = q.y - i.vy;
        const float uz = q.z - i.vz;
        const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, __builtin_fmaf(dx, dx, eps2)));
        const float rv = __builtin_fmaf(dz, uz, __builtin_fmaf(dy, uy, dx * ux));
        float rinv = __builtin_amdgcn_rsqf(r2);
        if (!SOFT) rinv = r2 > 0.0f ? rinv : 0.0f;
        const float rinv2 = rinv * rinv;
        float mr = q.w * rinv;
        if (MASK) mr = self ? 0.0f : mr;
        const float mr3 = mr * rinv2;
        const float t = -3.0f * (rv * rinv2);
        T.p += mr;
        T.ax = __builtin_fmaf(mr3, dx, T.ax);
        T.ay = __builtin_fmaf(mr3, dy, T.ay);
        T.az = __builtin_fmaf(mr3, dz, T.az);
        T.jx = __builtin_fmaf(mr3, __builtin_fmaf(t, dx, ux), T.jx);
        T.jy = __builtin_fmaf(mr3, __builtin_fmaf(t, dy, uy), T.jy);
        T.jz = __builtin_fmaf(mr3, __builtin_fmaf(t, dz, uz), T.jz);
    }
    __device__ static void fold(Sum &S, const Tile &T) {
        S.ax += (double)T.ax; S.ay += (double)T.ay; S.az += (double)T.az;
        S.jx += (double)T.jx; S.jy += (double)T.jy; S.jz += (double)T.jz;
        S.p += (double)T.p;
    }
    __device__ static Out7 out(const Sum &S) {
        return Out7{{S.ax, S.ay, S.az, S.jx, S.jy, S.jz, S.p}};
    }
    // S += the same record of the lane `off` away (xor), within a wave
    __device__ static void shfl_add(Sum &S, int off) {
        S.ax += __shfl_xor(S.ax, off, 64); S.ay += __shfl_xor(S.ay, off, 64);
        S.az += __shfl_xor(S.az, off, 64); S.jx += __shfl_xor(S.jx, off, 64);
        S.jy += __shfl_xor(S.jy, off, 64); S.jz += __shfl_xor(S.jz, off, 64);
        S.p += __shfl_xor(S.p, off, 64);
    }
};

// ------------------------------------------------------------------------------------------
// All-single interaction, the arithmetic of the paper's GPU kernel (Sec. Mapping and the
// force routine of Appendix A): predicted positions, velocities and masses are rounded to
// float, separations are differences of float positions, and the sums over all j stay in
// float.  Prediction and correction remain FP64.  Kept as the paper-style accuracy reference;
// separations cancel digits here that the FP32 mode keeps.
// ------------------------------------------------------------------------------------------
struct ModeF32All {
    struct Args {
        const float4 *pm;  // x, y, z, m
        const float4 *vv;  // vx, vy, vz, 0
        float eps2;
    };
    struct I {
        float x, y, z, vx, vy, vz, m;
    };
    struct Smem {
        float4 pm[TJ], vv[TJ];
    };
    struct Tile {
        float ax, ay, az, jx, jy, jz, p;
    };
    using Sum = Tile;

    __device__ static I load_i(const Args &a, int g) {
        const float4 q = a.pm[g], w = a.vv[g];
        return I{q.x, q.y, q.z, w.x, w.y, w.z, q.w};
    }
    __device__ static void stage(const Args &a, Smem &s, int t, int j, int n) {
        if (j < n) {
            s.pm[t] = a.pm[j]; s.vv[t] = a.vv[j];
        } else {  // padding: zero mass contributes nothing
            s.pm[t] = make_float4(0.f, 0.f, 0.f, 0.f); s.vv[t] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
    }
    __device__ static Tile tile_zero() { return Tile{0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f}; }
    __device__ static Sum sum_zero() { return tile_zero(); }
    __device__ static I make_i(const double xp[3], const double vp[3], double m) {
        return I{(float)xp[0], (float)xp[1], (float)xp[2], (float)vp[0], (float)vp[1],
                 (float)vp[2], (float)m};
    }
    __device__ static void put(Smem &s, int t, const double xp[3], const double vp[3], double m) {
        s.pm[t] = make_float4((float)xp[0], (float)xp[1], (float)xp[2], (float)m);
        s.vv[t] = make_float4((float)vp[0], (float)vp[1], (float)vp[2], 0.f);
    }

    struct J {
        float4 pm, vv;
    };
    __device__ static __forceinline__ J load_j(const Args &a, int j) {
        return J{uload(a.pm, j), uload(a.vv, j)};
    }
    template <bool SOFT, bool MASK = false>
    __device__ static __forceinline__ void interact(const I &i, const Smem &s, int jj, float eps2,
                                                    Tile &T, bool self = false) {
        pair<SOFT, MASK>(i, J{s.pm[jj], s.vv[jj]}, eps2, T, self);
    }
    template <bool SOFT, bool MASK = false>
    __device__ static __forceinline__ void pair(const I &i, const J &j, float eps2, Tile &T,
                                                bool self = false) {
        const float4 q = j.pm, w = j.vv;
        const float dx = q.x - i.x, dy = q.y - i.y, dz = q.z - i.z;
        const float ux = w.x - i.vx, uy = w.y - i.vy, uz = w.z - i.vz;
        const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, __builtin_fmaf(dx, dx, eps2)));
        const float rv = __builtin_fmaf(dz, uz, __builtin_fmaf(dy, uy, dx * ux));
        float rinv = __builtin_amdgcn_rsqf(r2);
        if (!SOFT) rinv = r2 > 0.0f ? rinv : 0.0f;
        const float rinv2 = rinv * rinv;
        float mr = q.w * rinv;
        if (MASK) mr = self ? 0.0f : mr;
        const float mr3 = mr * rinv2;
        const float t = -3.0f * (rv * rinv2);
        T.p += mr;
        T.ax = __builtin_fmaf(mr3, dx, T.ax);
        T.ay = __builtin_fmaf(mr3, dy, T.ay);
        T.az = __builtin_fmaf(mr3, dz, T.az);
        T.jx = __builtin_fmaf(mr3, __builtin_fmaf(t, dx, ux), T.jx);
        T.jy = __builtin_fmaf(mr3, __builtin_fmaf(t, dy, uy), T.jy);
        T.jz = __builtin_fmaf(mr3, __builtin_fmaf(t, dz, uz), T.jz);
    }
    __device__ static void fold(Sum &S, const Tile &T) {
        S.ax += T.ax; S.ay += T.ay; S.az += T.az;
        S.jx += T.jx; S.jy += T.jy; S.jz += T.jz;
        S.p += T.p;
    }
    __device__ static Out7 out(const Sum &S) {
        return Out7{{(double)S.ax, (double)S.ay, (double)S.az, (double)S.jx, (double)S.jy,
                     (double)S.jz, (double)S.p}};
    }
    __device__ static void shfl_add(Sum &S, int off) {
        S.ax += __shfl_xor(S.ax, off, 64); S.ay += __shfl_xor(S.ay, off, 64);
        S.az += __shfl_xor(S.az, off, 64); S.jx += __shfl_xor(S.jx, off, 64);
        S.jy += __shfl_xor(S.jy, off, 64); S.jz += __shfl_xor(S.jz, off, 64);
        S.p += __shfl_xor(S.p, off, 64);
    }
};

// ------------------------------------------------------------------------------------------
// Order-independent single precision, in the spirit of the 64-bit fixed-point accumulation of
// the GRAPE-6 pipelines the paper compares against (Sec. Results, accuracy measurements).  The
// interaction is the FP32 mode's; float sums run over aligned sub-blocks of FOLD = 64 j, and
// each sub-block sum is added into int64 accumulators in fixed point (scale 2^F per quantity).
// Integer addition is exact and associative, and a sub-block's float sum depends only on which
// j it holds, so the result is bitwise the same for any j-split, i-per-lane, unroll, work-item
// count or lane split.  Fixed-point steps: acc and pot 2^-44 (range +-2^19), jerk 2^-42
// (+-2^21).  With total mass 1 a softened pull is at most 0.385/eps^2 and a potential 1/eps,
// inside the range for eps >= 1e-3; the steps keep the rounding of N/64 sub-block conversions
// (about 2^-44 sqrt(N/64) absolute) far below single-precision error also for the small
// accelerations and jerks of halo particles.  A sub-block sum outside the range or an
// overflowing accumulator poisons the record, which comes out as NaN (reported as a
// non-finite force).
// ------------------------------------------------------------------------------------------
struct ModeF32Fixed : ModeF32 {
    static constexpr int F_ACC = 44, F_JERK = 42, F_POT = 44;
    struct Sum {
        int64_t ax, ay, az, jx, jy, jz, p;
        int32_t bad;
    };
    __device__ static Sum sum_zero() { return Sum{0, 0, 0, 0, 0, 0, 0, 0}; }
    __device__ static __forceinline__ int64_t fix(float x, int F, int32_t &bad) {
        const double d = __builtin_ldexp((double)x, F);  // exact
        const bool ok = __builtin_fabs(d) < 0x1p62;      // false for NaN too
        bad |= !ok;
        return ok ? (int64_t)__builtin_rint(d) : 0;
    }
    __device__ static __forceinline__ void add(int64_t &s, int64_t v, int32_t &bad) {
        const int64_t r = (int64_t)((uint64_t)s + (uint64_t)v);
        bad |= (int32_t)((uint64_t)((s ^ r) & (v ^ r)) >> 63);
        s = r;
    }
    __device__ static void fold(Sum &S, const Tile &T) {
        add(S.ax, fix(T.ax, F_ACC, S.bad), S.bad);
        add(S.ay, fix(T.ay, F_ACC, S.bad), S.bad);
        add(S.az, fix(T.az, F_ACC, S.bad), S.bad);
        add(S.jx, fix(T.jx, F_JERK, S.bad), S.bad);
        add(S.jy, fix(T.jy, F_JERK, S.bad), S.bad);
        add(S.jz, fix(T.jz, F_JERK, S.bad), S.bad);
        add(S.p, fix(T.p, F_POT, S.bad), S.bad);
    }
    __device__ static Out7 out(const Sum &S) {
        if (S.bad) {
            const double nan = __builtin_nan("");
            return Out7{{nan, nan, nan, nan, nan, nan, nan}};
        }
        return Out7{{__builtin_ldexp((double)S.ax, -F_ACC), __builtin_ldexp((double)S.ay, -F_ACC),
                     __builtin_ldexp((double)S.az, -F_ACC), __builtin_ldexp((double)S.jx, -F_JERK),
                     __builtin_ldexp((double)S.jy, -F_JERK), __builtin_ldexp((double)S.jz, -F_JERK),
                     __builtin_ldexp((double)S.p, -F_POT)}};
    }
    // K > 1: the raw integers go to the partial planes (INT64_MIN marks a poisoned record)
    __device__ static void store_raw(double *base, int64_t P, const Sum &S) {
        const int64_t v[7] = {S.ax, S.ay, S.az, S.jx, S.jy, S.jz, S.p};
#pragma unroll
        for (int c = 0; c < 7; ++c)
            base[(int64_t)c * P] = __longlong_as_double(S.bad ? INT64_MIN : (long long)v[c]);
    }
    __device__ static void shfl_add(Sum &S, int off) {
        add(S.ax, __shfl_xor(S.ax, off, 64), S.bad); add(S.ay, __shfl_xor(S.ay, off, 64), S.bad);
        add(S.az, __shfl_xor(S.az, off, 64), S.bad); add(S.jx, __shfl_xor(S.jx, off, 64), S.bad);
        add(S.jy, __shfl_xor(S.jy, off, 64), S.bad); add(S.jz, __shfl_xor(S.jz, off, 64), S.bad);
        add(S.p, __shfl_xor(S.p, off, 64), S.bad);
        S.bad |= __shfl_xor(S.bad, off, 64);
    }
};

// ------------------------------------------------------------------------------------------
// Double-single interaction: every operation in float-float arithmetic; tile sums folded into
// outer sums with the accurate addition.
// ------------------------------------------------------------------------------------------
struct ModeDS {
    struct Args {
        const float4 *q0;  // x_hi, y_hi, z_hi, m_hi
        const float4 *q1;  // x_lo, y_lo, z_lo, m_lo
        const float4 *q2;  // vx_hi, vy_hi, vz_hi, 0
        const float4 *q3;  // vx_lo, vy_lo, vz_lo, 0
        ds eps2;
    };
    struct I {
        ds x, y, z, vx, vy, vz, m;
    };
    struct Smem {
        float4 q0[TJ], q1[TJ], q2[TJ], q3[TJ];
    };
    struct Tile {
        ds ax, ay, az, jx, jy, jz, p;
    };
    using Sum = Tile;

    __device__ static I load_i(const Args &a, int g) {
        const float4 h = a.q0[g], l = a.q1[g], vh = a.q2[g], vl = a.q3[g];
        return I{ds{h.x, l.x}, ds{h.y, l.y}, ds{h.z, l.z}, ds{vh.x, vl.x}, ds{vh.y, vl.y},
                 ds{vh.z, vl.z}, ds{h.w, l.w}};
    }
    __device__ static void stage(const Args &a, Smem &s, int t, int j, int n) {
        if (j < n) {
            s.q0[t] = a.q0[j]; s.q1[t] = a.q1[j]; s.q2[t] = a.q2[j]; s.q3[t] = a.q3[j];
        } else {
            const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
            s.q0[t] = z; s.q1[t] = z; s.q2[t] = z; s.q3[t] = z;
        }
    }
    __device__ static Tile tile_zero() {
        const ds z{0.f, 0.f};
        return Tile{z, z, z, z, z, z, z};
    }
    __device__ static Sum sum_zero() { return tile_zero(); }
    __device__ static I make_i(const double xp[3], const double vp[3], double m) {
        return I{ds_from_double(xp[0]), ds_from_double(xp[1]), ds_from_double(xp[2]),
                 ds_from_double(vp[0]), ds_from_double(vp[1]), ds_from_double(vp[2]),
                 ds_from_double(m)};
    }
    __device__ static void put(Smem &s, int t, const double xp[3], const double vp[3], double m) {
        const ds X = ds_from_double(xp[0]), Y = ds_from_double(xp[1]), Z = ds_from_double(xp[2]);
        const ds VX = ds_from_double(vp[0]), VY = ds_from_double(vp[1]), VZ = ds_from_double(vp[2]);
        const ds M = ds_from_double(m);
        s.q0[t] = make_float4(X.hi, Y.hi, Z.hi, M.hi);
        s.q1[t] = make_float4(X.lo, Y.lo, Z.lo, M.lo);
        s.q2[t] = make_float4(VX.hi, VY.hi, VZ.hi, 0.f);
        s.q3[t] = make_float4(VX.lo, VY.lo, VZ.lo, 0.f);
    }

    struct J {
        float4 h, l, vh, vl;
    };
    __device__ static __forceinline__ J load_j(const Args &a, int j) {
        return J{uload(a.q0, j), uload(a.q1, j), uload(a.q2, j), uload(a.q3, j)};
    }
    template <bool SOFT, bool MASK = false>
    __device__ static __forceinline__ void interact(const I &i, const Smem &s, int jj, ds eps2,
                                                    Tile &T, bool self = false) {
        pair<SOFT, MASK>(i, J{s.q0[jj], s.q1[jj], s.q2[jj], s.q3[jj]}, eps2, T, self);
    }
    template <bool SOFT, bool MASK = false>
    __device__ static __forceinline__ void pair(const I &i, const J &j, ds eps2, Tile &T,
                                                bool self = false) {
        const float4 h = j.h, l = j.l, vh = j.vh, vl = j.vl;
        // separations: the high parts' difference is exact (two_sum), the low parts' adds one
        // rounding of about 2^-48 |x|; products skip their own renormalisation (the additions
        // renormalise)
        const ds dx = ds_add_sloppy(ds{h.x, l.x}, ds_neg(i.x));
        const ds dy = ds_add_sloppy(ds{h.y, l.y}, ds_neg(i.y));
        const ds dz = ds_add_sloppy(ds{h.z, l.z}, ds_neg(i.z));
        const ds ux = ds_add_sloppy(ds{vh.x, vl.x}, ds_neg(i.vx));
        const ds uy = ds_add_sloppy(ds{vh.y, vl.y}, ds_neg(i.vy));
        const ds uz = ds_add_sloppy(ds{vh.z, vl.z}, ds_neg(i.vz));
        const ds r2 = ds_add_sloppy(
            ds_add_sloppy(ds_add_sloppy(eps2, ds_sqr_raw(dx)), ds_sqr_raw(dy)), ds_sqr_raw(dz));
        const ds rv = ds_add_sloppy(ds_add_sloppy(ds_mul_raw(dx, ux), ds_mul_raw(dy, uy)),
                                    ds_mul_raw(dz, uz));
        ds rinv = ds_rsqrt(r2);
        if (!SOFT && !(r2.hi > 0.0f)) rinv = ds{0.f, 0.f};
        const ds rinv2 = ds_sqr_raw(rinv);
        ds mr = ds_mul_raw(ds{h.w, l.w}, rinv);
        if (MASK) mr = ds{self ? 0.0f : mr.hi, self ? 0.0f : mr.lo};
        const ds mr3 = ds_mul_raw(mr, rinv2);
        const ds t = ds_mul_f_raw(ds_mul_raw(rv, rinv2), -3.0f);
        T.p = ds_add_sloppy(T.p, mr);
        T.ax = ds_add_sloppy(T.ax, ds_mul_raw(mr3, dx));
        T.ay = ds_add_sloppy(T.ay, ds_mul_raw(mr3, dy));
        T.az = ds_add_sloppy(T.az, ds_mul_raw(mr3, dz));
        T.jx = ds_add_sloppy(T.jx, ds_mul_raw(mr3, ds_add_sloppy(ux, ds_mul_raw(t, dx))));
        T.jy = ds_add_sloppy(T.jy, ds_mul_raw(mr3, ds_add_sloppy(uy, ds_mul_raw(t, dy))));
        T.jz = ds_add_sloppy(T.jz, ds_mul_raw(mr3, ds_add_sloppy(uz, ds_mul_raw(t, dz))));
    }
    __device__ static void fold(Sum &S, const Tile &T) {
        S.ax = ds_add(S.ax, T.ax); S.ay = ds_add(S.ay, T.ay); S.az = ds_add(S.az, T.az);
        S.jx = ds_add(S.jx, T.jx); S.jy = ds_add(S.jy, T.jy); S.jz = ds_add(S.jz, T.jz);
        S.p = ds_add(S.p, T.p);
    }
    __device__ static Out7 out(const Sum &S) {
        return Out7{{ds_to_double(S.ax), ds_to_double(S.ay), ds_to_double(S.az),
                     ds_to_double(S.jx), ds_to_double(S.jy), ds_to_double(S.jz),
                     ds_to_double(S.p)}};
    }
    __device__ static ds shfl_ds(ds a, int off) {
        return ds{__shfl_xor(a.hi, off, 64), __shfl_xor(a.lo, off, 64)};
    }
    __device__ static void shfl_add(Sum &S, int off) {
        S.ax = ds_add(S.ax, shfl_ds(S.ax, off)); S.ay = ds_add(S.ay, shfl_ds(S.ay, off));
        S.az = ds_add(S.az, shfl_ds(S.az, off)); S.jx = ds_add(S.jx, shfl_ds(S.jx, off));
        S.jy = ds_add(S.jy, shfl_ds(S.jy, off)); S.jz = ds_add(S.jz, shfl_ds(S.jz, off));
        S.p = ds_add(S.p, shfl_ds(S.p, off));
    }
};

// ------------------------------------------------------------------------------------------
// FP64 interaction: IEEE double throughout; s^(-1/2) from the hardware estimate refined by one
// correction step of third order, y = y0 (1 + r/2 + 3 r^2/8) with r = 1 - s y0^2 (relative
// error about 5/16 of the estimate's cubed).
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ double rsqrt_f64(double s) {
    const double y = __builtin_amdgcn_rsq(s);
    const double r = __builtin_fma(-(s * y), y, 1.0);
    return __builtin_fma(y * r, __builtin_fma(0.375, r, 0.5), y);
}

struct ModeF64 {
    struct Args {
        const double *px, *py, *pz, *pm, *vx, *vy, *vz;
        double eps2;
    };
    struct I {
        double x, y, z, vx, vy, vz, m;
    };
    // one 64-byte record per staged j (a single LDS address for all seven values)
    struct Rec {
        double x, y, z, m, vx, vy, vz, pad;
    };
    struct Smem {
        Rec r[TJ];
    };
    struct Tile {
        double ax, ay, az, jx, jy, jz, p;
    };
    using Sum = Tile;

    __device__ static I load_i(const Args &a, int g) {
        return I{a.px[g], a.py[g], a.pz[g], a.vx[g], a.vy[g], a.vz[g], a.pm[g]};
    }
    __device__ static void stage(const Args &a, Smem &s, int t, int j, int n) {
        const bool ok = j < n;
        s.r[t] = Rec{ok ? a.px[j] : 0.0, ok ? a.py[j] : 0.0, ok ? a.pz[j] : 0.0,
                     ok ? a.pm[j] : 0.0, ok ? a.vx[j] : 0.0, ok ? a.vy[j] : 0.0,
                     ok ? a.vz[j] : 0.0, 0.0};
    }
    __device__ static Tile tile_zero() { return Tile{0., 0., 0., 0., 0., 0., 0.}; }
    __device__ static Sum sum_zero() { return tile_zero(); }
    __device__ static I make_i(const double xp[3], const double vp[3], double m) {
        return I{xp[0], xp[1], xp[2], vp[0], vp[1], vp[2], m};
    }
    __device__ static void put(Smem &s, int t, const double xp[3], const double vp[3], double m) {
        s.r[t] = Rec{xp[0], xp[1], xp[2], m, vp[0], vp[1], vp[2], 0.0};
    }

    struct J {
        double x, y, z, m, vx, vy, vz;
    };
    __device__ static __forceinline__ J load_j(const Args &a, int j) {
        return J{uload(a.px, j), uload(a.py, j), uload(a.pz, j), uload(a.pm, j),
                 uload(a.vx, j), uload(a.vy, j), uload(a.vz, j)};
    }
    template <bool SOFT, bool MASK = false>
    __device__ static __forceinline__ void interact(const I &i, const Smem &s, int jj, double eps2,
                                                    Tile &T, bool self = false) {
        const Rec &q = s.r[jj];
        pair<SOFT, MASK>(i, J{q.x, q.y, q.z, q.m, q.vx, q.vy, q.vz}, eps2, T, self);
    }
    template <bool SOFT, bool MASK = false>
    __device__ static __forceinline__ void pair(const I &i, const J &j, double eps2, Tile &T,
                                                bool self = false) {
        const double dx = j.x - i.x, dy = j.y - i.y, dz = j.z - i.z;
        const double ux = j.vx - i.vx, uy = j.vy - i.vy, uz = j.vz - i.vz;
        const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, __builtin_fma(dx, dx, eps2)));
        const double rv = __builtin_fma(dz, uz, __builtin_fma(dy, uy, dx * ux));
        double rinv = rsqrt_f64(r2);
        if (!SOFT) rinv = r2 > 0.0 ? rinv : 0.0;
        const double rinv2 = rinv * rinv;
        double mr = j.m * rinv;
        if (MASK) mr = self ? 0.0 : mr;
        const double mr3 = mr * rinv2;
        const double t = -3.0 * (rv * rinv2);
        T.p += mr;
        T.ax = __builtin_fma(mr3, dx, T.ax);
        T.ay = __builtin_fma(mr3, dy, T.ay);
        T.az = __builtin_fma(mr3, dz, T.az);
        T.jx = __builtin_fma(mr3, __builtin_fma(t, dx, ux), T.jx);
        T.jy = __builtin_fma(mr3, __builtin_fma(t, dy, uy), T.jy);
        T.jz = __builtin_fma(mr3, __builtin_fma(t, dz, uz), T.jz);
    }
    __device__ static void fold(Sum &S, const Tile &T) {
        S.ax += T.ax; S.ay += T.ay; S.az += T.az; S.jx += T.jx; S.jy += T.jy; S.jz += T.jz;
        S.p += T.p;
    }
    __device__ static Out7 out(const Sum &S) {
        return Out7{{S.ax, S.ay, S.az, S.jx, S.jy, S.jz, S.p}};
    }
    __device__ static void shfl_add(Sum &S, int off) {
        S.ax += __shfl_xor(S.ax, off, 64); S.ay += __shfl_xor(S.ay, off, 64);
        S.az += __shfl_xor(S.az, off, 64); S.jx += __shfl_xor(S.jx, off, 64);
        S.jy += __shfl_xor(S.jy, off, 64); S.jz += __shfl_xor(S.jz, off, 64);
        S.p += __shfl_xor(S.p, off, 64);
    }
};

__device__ __forceinline__ bool finite7(const Out7 &o) {
    bool ok = true;
#pragma unroll
    for (int c = 0; c < 7; ++c) ok = ok && __builtin_isfinite(o.v[c]);
    return ok;
}

template <class M> struct EpsOf;
template <> struct EpsOf<ModeF32> { using T = float; };
template <> struct EpsOf<ModeDS> { using T = ds; };
template <> struct EpsOf<ModeF64> { using T = double; };
template <> struct EpsOf<ModeF32All> { using T = float; };
template <> struct EpsOf<ModeF32Fixed> { using T = float; };

// How a mode folds its sums: every FOLD j of a tile (TJ: once per tile), and whether the sums
// are fixed-point integers (then at most TJ / FOLD lanes may share an i-particle).
// SCALAR_J: whole blocks read the j-records with scalar loads (measured faster for the float
// modes: 611 against 664 ms for the FP32 full force at N = 2^20) or from LDS tiles (FP64,
// whose 56-byte record made the scalar path slower: 1.71 against 1.34 s).
template <class M> struct ModeTraits {
    static constexpr int FOLD = TJ;
    static constexpr bool FIXED = false;
    static constexpr bool SCALAR_J = true;
};
template <> struct ModeTraits<ModeF32Fixed> {
    static constexpr int FOLD = 64;
    static constexpr bool FIXED = true;
    static constexpr bool SCALAR_J = true;
};
template <> struct ModeTraits<ModeF64> {
    static constexpr int FOLD = TJ;
    static constexpr bool FIXED = false;
    static constexpr bool SCALAR_J = false;
};

// Final sums of row q of a work item's j-range ks: straight to the outputs when K == 1,
// else to partial plane ks.  The potential sum is negated here (for fixed-point sums, whose
// partial planes hold the raw integers, in the reduction).
template <class M>
__device__ __forceinline__ void store_result(const ForceCommon &fc, const ForcePlan &pl,
                                             int32_t ks, int32_t q, const typename M::Sum &S) {
    double *base = fc.partial + (int64_t)ks * 7 * pl.P + q;
    if constexpr (ModeTraits<M>::FIXED) {
        if (pl.K > 1) {
            M::store_raw(base, pl.P, S);
            return;
        }
    }
    Out7 o = M::out(S);
    o.v[6] = -o.v[6];
    if (pl.K == 1) {
        if (fc.ctl && !finite7(o)) fc.ctl->flag_nonfinite = 1;
        fc.acc[0 * (int64_t)fc.ld + q] = o.v[0];
        fc.acc[1 * (int64_t)fc.ld + q] = o.v[1];
        fc.acc[2 * (int64_t)fc.ld + q] = o.v[2];
        fc.jerk[0 * (int64_t)fc.ld + q] = o.v[3];
        fc.jerk[1 * (int64_t)fc.ld + q] = o.v[4];
        fc.jerk[2 * (int64_t)fc.ld + q] = o.v[5];
        fc.pot[q] = o.v[6];
    } else {
#pragma unroll
        for (int c = 0; c < 7; ++c) base[(int64_t)c * pl.P] = o.v[c];
    }
}

// One staged tile for a lane that takes the j-slots slice, slice + Sl, ... (Sl = 1: all):
// float-mode tile sums folded once per tile, fixed-point sums once per FOLD-j sub-block (lanes
// then take whole sub-blocks).  MASK: the slot `own` of the tile (if any) is the lane's own
// particle and adds nothing.
template <class M, int UNR, bool SOFT, bool MASK>
__device__ __forceinline__ void sums_tile(const typename M::I &ii, const typename M::Smem &sm,
                                          int32_t slice, int32_t Sl, int32_t own,
                                          typename EpsOf<M>::T eps2, typename M::Sum &S) {
    if constexpr (ModeTraits<M>::FOLD == TJ) {
        typename M::Tile T = M::tile_zero();
#pragma unroll UNR
        for (int jj = slice; jj < TJ; jj += Sl)
            M::template interact<SOFT, MASK>(ii, sm, jj, eps2, T, jj == own);
        M::fold(S, T);
    } else {  // lanes take whole sub-blocks of FOLD j (Sl <= TJ / FOLD)
        constexpr int FOLD = ModeTraits<M>::FOLD;
        for (int b = slice; b < TJ / FOLD; b += Sl) {
            typename M::Tile T = M::tile_zero();
#pragma unroll UNR
            for (int jj = b * FOLD; jj < (b + 1) * FOLD; ++jj)
                M::template interact<SOFT, MASK>(ii, sm, jj, eps2, T, jj == own);
            M::fold(S, T);
        }
    }
}

// Small i-lists: S adjacent lanes share one i-particle, lane `slice` of the group takes the
// j-particles slice, slice + S, ... of every staged tile, and the S partial sums are combined
// by xor-shuffles within the wave (a fixed order) before the result is stored.
template <class M, int UNR, bool SOFT>
__device__ void force_items_split(const typename M::Args &pa, const ForceCommon &fc,
                                  const ForcePlan &pl, typename M::Smem &sm, int32_t n_i,
                                  typename EpsOf<M>::T eps2) {
    const int32_t Sl = pl.S;
    const int32_t slice = (int32_t)threadIdx.x % Sl;
    for (int32_t w = blockIdx.x; w < pl.items; w += gridDim.x) {
        const int32_t iblk = w / pl.K, ks = w - (w / pl.K) * pl.K;
        const int32_t q = iblk * pl.ib + (int32_t)threadIdx.x / Sl;
        const int32_t g = q < n_i ? (fc.ilist ? fc.ilist[q] : q) : 0;
        const int32_t own = q < n_i ? g : -1;  // the i-particle's own j-slot (none on padding)
        const typename M::I ii = M::load_i(pa, g);
        typename M::Sum S = M::sum_zero();
        const int32_t t0 = ks * pl.tps;
        const int32_t t1 = t0 + pl.tps < pl.ntiles ? t0 + pl.tps : pl.ntiles;
        for (int32_t t = t0; t < t1; ++t) {
            __syncthreads();
            M::stage(pa, sm, threadIdx.x, t * TJ + (int32_t)threadIdx.x, fc.n);
            __syncthreads();
            // a tile holding a lane's own slot takes the masked loop (wave-uniform branch)
            const int32_t rel = own - t * TJ;
            if (SOFT && __ballot((uint32_t)rel < (uint32_t)TJ) != 0) {
                sums_tile<M, UNR, SOFT, true>(ii, sm, slice, Sl, rel, eps2, S);
            } else {
                sums_tile<M, UNR, SOFT, false>(ii, sm, slice, Sl, rel, eps2, S);
            }
        }
        for (int off = Sl >> 1; off > 0; off >>= 1) M::shfl_add(S, off);
        if (slice == 0 && q < n_i) store_result<M>(fc, pl, ks, q, S);
    }
}

// Sums of the IPL i-particles of a work-item over the j-tiles [t0, t1): the j-records read
// once per wave with scalar loads (every lane takes the same j).  The latency of each load is
// exposed to its wave, so the launch takes this path only for items of at least
// ForceCommon::scalar_min tiles (chosen per launch class by measurement).

// Sums over j in [ja, je) with scalar j-loads; MASK: some lane's own slot own[p] lies inside.
template <class M, int IPL, int UNR, bool SOFT, bool MASK>
__device__ __forceinline__ void sums_scalar_run(const typename M::Args &pa, int32_t ja, int32_t je,
                                                const typename M::I (&ii)[IPL],
                                                const int32_t (&own)[IPL],
                                                typename M::Tile (&T)[IPL],
                                                typename EpsOf<M>::T eps2) {
#pragma unroll UNR
    for (int32_t j = ja; j < je; ++j) {
        const typename M::J jr = M::load_j(pa, j);
#pragma unroll
        for (int p = 0; p < IPL; ++p) M::template pair<SOFT, MASK>(ii[p], jr, eps2, T[p], j == own[p]);
    }
}

template <class M, int IPL, int UNR, bool SOFT>
__device__ __forceinline__ void block_sums_scalar(const typename M::Args &pa, int32_t n, int32_t t0,
                                                  int32_t t1, const typename M::I (&ii)[IPL],
                                                  const int32_t (&own)[IPL],
                                                  typename M::Sum (&S)[IPL],
                                                  typename EpsOf<M>::T eps2) {
    constexpr int FOLD = ModeTraits<M>::FOLD;
    for (int32_t t = t0; t < t1; ++t) {
        const int32_t j0 = t * TJ;
        const int32_t jn = n - j0 < TJ ? n - j0 : TJ;
        for (int32_t jb = 0; jb < jn; jb += FOLD) {
            // wave-uniform bounds kept in scalar registers
            const int32_t ja = __builtin_amdgcn_readfirstlane(j0 + jb);
            const int32_t je = __builtin_amdgcn_readfirstlane(j0 + (jb + FOLD < jn ? jb + FOLD : jn));
            typename M::Tile T[IPL];
#pragma unroll
            for (int p = 0; p < IPL; ++p) T[p] = M::tile_zero();
            // a run holding some lane's own slot takes the masked loop (wave-uniform branch)
            bool hit = false;
#pragma unroll
            for (int p = 0; p < IPL; ++p) hit = hit || (uint32_t)(own[p] - ja) < (uint32_t)(je - ja);
            if (SOFT && __ballot(hit) != 0)
                sums_scalar_run<M, IPL, UNR, SOFT, true>(pa, ja, je, ii, own, T, eps2);
            else
                sums_scalar_run<M, IPL, UNR, SOFT, false>(pa, ja, je, ii, own, T, eps2);
#pragma unroll
            for (int p = 0; p < IPL; ++p) M::fold(S[p], T[p]);
        }
    }
}

// The same sums from LDS tiles staged by the whole workgroup (one j per work-item, loads
// coalesced); every lane then reads each staged j (a broadcast).  Padding j past n has zero
// mass and adds exact zeros, so both paths give bitwise the same sums.
template <class M, int IPL, int UNR, bool SOFT, bool MASK>
__device__ __forceinline__ void sums_lds_run(const typename M::Smem &sm, int jb, int je,
                                             const typename M::I (&ii)[IPL],
                                             const int32_t (&rel)[IPL], typename M::Tile (&T)[IPL],
                                             typename EpsOf<M>::T eps2) {
#pragma unroll UNR
    for (int jj = jb; jj < je; ++jj) {
#pragma unroll
        for (int p = 0; p < IPL; ++p)
            M::template interact<SOFT, MASK>(ii[p], sm, jj, eps2, T[p], jj == rel[p]);
    }
}

template <class M, int IPL, int UNR, bool SOFT>
__device__ __forceinline__ void block_sums_lds(const typename M::Args &pa, int32_t n,
                                               typename M::Smem &sm, int32_t t0, int32_t t1,
                                               const typename M::I (&ii)[IPL],
                                               const int32_t (&own)[IPL],
                                               typename M::Sum (&S)[IPL],
                                               typename EpsOf<M>::T eps2) {
    constexpr int FOLD = ModeTraits<M>::FOLD;
    for (int32_t t = t0; t < t1; ++t) {
        __syncthreads();
        M::stage(pa, sm, threadIdx.x, t * TJ + (int32_t)threadIdx.x, n);
        __syncthreads();
        int32_t rel[IPL];
#pragma unroll
        for (int p = 0; p < IPL; ++p) rel[p] = own[p] - t * TJ;
        for (int jb = 0; jb < TJ; jb += FOLD) {
            typename M::Tile T[IPL];
#pragma unroll
            for (int p = 0; p < IPL; ++p) T[p] = M::tile_zero();
            bool hit = false;
#pragma unroll
            for (int p = 0; p < IPL; ++p) hit = hit || (uint32_t)(rel[p] - jb) < (uint32_t)FOLD;
            if (SOFT && __ballot(hit) != 0)
                sums_lds_run<M, IPL, UNR, SOFT, true>(sm, jb, jb + FOLD, ii, rel, T, eps2);
            else
                sums_lds_run<M, IPL, UNR, SOFT, false>(sm, jb, jb + FOLD, ii, rel, T, eps2);
#pragma unroll
            for (int p = 0; p < IPL; ++p) M::fold(S[p], T[p]);
        }
    }
}

// ------------------------------------------------------------------------------------------
// The force kernel.  Each workgroup takes work items (i-block, j-range); each work-item holds
// IPL i-particles in registers.  On the whole-block path every lane of a wave takes the same j
// at the same time: on long j-ranges the float modes read each j-record once per wave with
// scalar loads (no LDS, no barriers); FP64, and every mode on short j-ranges, stage TJ
// j-particles at a time in LDS and every lane reads each staged j (a broadcast).  The j-loop
// is unrolled UNR times.  The tile sums are folded into the outer sums every FOLD j counted
// from the start of each TJ-tile (the same j-indices on every path, so the path never changes
// a result).  Short lists take the lane split, which stages TJ j-particles at a time in LDS
// (force_items_split).
// K == 1: results go straight to acc/jerk/pot; K > 1: to the partial planes for
// force_reduce.  The potential sum is negated on output.
// The self pair j = i is excluded (Eq. Force sums over j != i): every run of j-slots (a tile, or
// a fixed-point sub-block) that holds some lane's own particle is taken by a masked copy of the
// loop in which that slot adds nothing; all other runs take the unmasked loop.  (With eps > 0
// the self slot would add m_i / eps to the potential's float tile sum, whose rounding would
// then be relative to m_i / eps rather than to the potential; with eps = 0 every pair at zero
// separation is skipped anyway.)
// ------------------------------------------------------------------------------------------
// CLS only separates the symbols of full-force launches (0) and block-step launches (1) so that
// profilers report the two launch classes apart; the code is the same.
template <class M, int IPL, int UNR, bool SOFT, int CLS>
__global__ void __launch_bounds__(WG) force_kernel(typename M::Args pa, ForceCommon fc) {
    __shared__ typename M::Smem sm;
    int32_t n_i = fc.n_i_max;
    if (fc.n_i_dev) {
        const int32_t d = *fc.n_i_dev;
        n_i = d < n_i ? d : n_i;
    }
    if (n_i <= 0) return;
    const ForcePlan pl = make_plan(n_i, fc.n, WG * IPL, fc.target, fc.kmax, fc.smax);
    const auto eps2 = pa.eps2;
    if (pl.S > 1) {
        force_items_split<M, UNR, SOFT>(pa, fc, pl, sm, n_i, eps2);
        return;
    }
    // XCD-aware order: workgroups are dealt to the chip's 8 XCDs round-robin, so with a grid
    // that is a multiple of 8, XCD x runs the workgroups x, x + 8, ...; they take the x-th
    // eighth of the items in (j-range major, i-block minor) order, and the workgroups resident
    // on one XCD at a time share few j-ranges, which its own L2 then holds.  Any other grid
    // takes the items in plain order.  Items are independent: the order never changes a result.
    const int32_t nx = (gridDim.x & 7) == 0 ? 8 : 1;
    const int32_t xcd = (int32_t)blockIdx.x % nx;
    const int32_t v_end = (int32_t)(((int64_t)pl.items * (xcd + 1)) / nx);
    const int32_t v_step = (int32_t)gridDim.x / nx;
    for (int32_t v = (int32_t)(((int64_t)pl.items * xcd) / nx) + (int32_t)blockIdx.x / nx;
         v < v_end; v += v_step) {
        const int32_t ks = v / pl.n_iblk, iblk = v - ks * pl.n_iblk;
        int32_t q[IPL], own[IPL];
        typename M::I ii[IPL];
        typename M::Sum S[IPL];
#pragma unroll
        for (int p = 0; p < IPL; ++p) {
            q[p] = iblk * (WG * IPL) + p * WG + (int32_t)threadIdx.x;
            const int32_t g = q[p] < n_i ? (fc.ilist ? fc.ilist[q[p]] : q[p]) : 0;
            own[p] = q[p] < n_i ? g : -1;  // the i-particle's own j-slot (none on padding)
            ii[p] = M::load_i(pa, g);
            S[p] = M::sum_zero();
        }
        const int32_t t0 = ks * pl.tps;
        const int32_t t1 = t0 + pl.tps < pl.ntiles ? t0 + pl.tps : pl.ntiles;
        if constexpr (ModeTraits<M>::SCALAR_J) {
            if (pl.tps >= fc.scalar_min)
                block_sums_scalar<M, IPL, UNR, SOFT>(pa, fc.n, t0, t1, ii, own, S, eps2);
            else
                block_sums_lds<M, IPL, UNR, SOFT>(pa, fc.n, sm, t0, t1, ii, own, S, eps2);
        } else {
            block_sums_lds<M, IPL, UNR, SOFT>(pa, fc.n, sm, t0, t1, ii, own, S, eps2);
        }
#pragma unroll
        for (int p = 0; p < IPL; ++p)
            if (q[p] < n_i) store_result<M>(fc, pl, ks, q[p], S[p]);
    }
}

// Fixed-order sum over the K partial planes (deterministic; no atomics).
// One workgroup per (64 consecutive i-rows, one of the 7 sums): wave w adds the planes
// k = w, w + RW, w + 2 RW, ... (in four interleaved partial sums, so that four loads are in
// flight) and the RW wave sums are then added in wave order, so the result depends only on K,
// never on timing.  Consecutive lanes read consecutive rows of a plane.
constexpr int RW = 16;               // waves per reduce workgroup
constexpr int WG_REDUCE = 64 * RW;

// FIXED: the planes hold the raw int64 fixed-point sums of ModeF32Fixed; they are added as
// integers (exact), converted with the mode's scales and the potential negated.
template <bool FIXED>
__global__ void __launch_bounds__(WG_REDUCE) force_reduce(ForceCommon fc, int32_t ib) {
    __shared__ double part[RW][64];
    __shared__ int64_t ipart[FIXED ? RW : 1][64];
    __shared__ int32_t ibad[FIXED ? RW : 1][64];
    int32_t n_i = fc.n_i_max;
    if (fc.n_i_dev) {
        const int32_t d = *fc.n_i_dev;
        n_i = d < n_i ? d : n_i;
    }
    if (n_i <= 0) return;
    const ForcePlan pl = make_plan(n_i, fc.n, ib, fc.target, fc.kmax, fc.smax);
    if (pl.K == 1) return;
    const int32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int32_t units = ((n_i + 63) >> 6) * 7;
    for (int32_t u = blockIdx.x; u < units; u += gridDim.x) {
        const int32_t rb = u / 7, c = u - rb * 7;
        const int32_t q = rb * 64 + lane;
        const double *src = fc.partial + (int64_t)c * pl.P + q;
        if constexpr (FIXED) {
            int64_t s = 0;
            int32_t bad = 0;
            if (q < n_i) {
                for (int32_t k = w; k < pl.K; k += RW) {
                    const int64_t v = (int64_t)__double_as_longlong(src[(int64_t)k * 7 * pl.P]);
                    bad |= v == INT64_MIN;
                    ModeF32Fixed::add(s, v, bad);
                }
            }
            ipart[w][lane] = s;
            ibad[w][lane] = bad;
        } else {
            // four planes in flight per lane: planes k = w + RW (4 m + r) go to sum r, and the
            // four sums are added in the order 0..3 (the order depends only on K)
            double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
            if (q < n_i) {
                const int64_t st = (int64_t)RW * 7 * pl.P;
                int32_t k = w;
                for (; k + 3 * RW < pl.K; k += 4 * RW) {
                    const double *b = src + (int64_t)k * 7 * pl.P;
                    s0 += b[0]; s1 += b[st]; s2 += b[2 * st]; s3 += b[3 * st];
                }
                for (; k < pl.K; k += RW) s0 += src[(int64_t)k * 7 * pl.P];
            }
            part[w][lane] = ((s0 + s1) + s2) + s3;
        }
        __syncthreads();
        if (w == 0 && q < n_i) {
            double t;
            if constexpr (FIXED) {
                int64_t s = ipart[0][lane];
                int32_t bad = ibad[0][lane];
#pragma unroll
                for (int r = 1; r < RW; ++r) {
                    bad |= ibad[r][lane];
                    ModeF32Fixed::add(s, ipart[r][lane], bad);
                }
                const int F = c < 3 ? ModeF32Fixed::F_ACC : c < 6 ? ModeF32Fixed::F_JERK
                                                                  : ModeF32Fixed::F_POT;
                t = bad ? __builtin_nan("") : __builtin_ldexp((double)s, -F);
                if (c == 6) t = -t;
            } else {
                t = part[0][lane];
#pragma unroll
                for (int r = 1; r < RW; ++r) t += part[r][lane];
            }
            if (fc.ctl && !__builtin_isfinite(t)) fc.ctl->flag_nonfinite = 1;
            double *dst = c < 3 ? fc.acc + c * (int64_t)fc.ld
                        : c < 6 ? fc.jerk + (c - 3) * (int64_t)fc.ld : fc.pot;
            dst[q] = t;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------------------------
// Sec. 2 predictor (FP64) of all particles to time t, written as the j-particle stream.
// ------------------------------------------------------------------------------------------
struct StateView {
    const double *x, *v, *a, *k, *m;
    const int64_t *tick;
    int32_t n;
    double tick_len;
};

struct JStreamView {
    double *px, *py, *pz;  // F32 / F64
    float4 *vm;            // F32
    float4 *q0, *q1, *q2, *q3;  // DS
    double *pm, *vx, *vy, *vz;  // F64
};

__device__ __forceinline__ void predict_one(double D, double x, double v, double a, double k,
                                            double &xp, double &vp) {
    const double h = 0.5 * D;
    const double t = D * (1.0 / 3.0);
    // x + D (v + D/2 (a + D/3 k)) and v + D (a + D/2 k)
    xp = __builtin_fma(D, __builtin_fma(h, __builtin_fma(t, k, a), v), x);
    vp = __builtin_fma(D, __builtin_fma(h, k, a), v);
}

// Predict particle i to tick t and store it in the j-stream layout of MODE (0: FP32 and
// fixed-point, 1: double-single, 2: FP64, 3: all-single).
template <int MODE>
__device__ __forceinline__ void predict_store(const StateView &s, const JStreamView &js, int32_t i,
                                              int64_t t) {
    const int32_t n = s.n;
    const double D = (double)(t - s.tick[i]) * s.tick_len;
    double xp[3], vp[3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
        predict_one(D, s.x[c * (int64_t)n + i], s.v[c * (int64_t)n + i],
                    s.a[c * (int64_t)n + i], s.k[c * (int64_t)n + i], xp[c], vp[c]);
    const double m = s.m[i];
    if (MODE == 0) {
        js.px[i] = xp[0]; js.py[i] = xp[1]; js.pz[i] = xp[2];
        js.vm[i] = make_float4((float)vp[0], (float)vp[1], (float)vp[2], (float)m);
    } else if (MODE == 3) {
        js.q0[i] = make_float4((float)xp[0], (float)xp[1], (float)xp[2], (float)m);
        js.q1[i] = make_float4((float)vp[0], (float)vp[1], (float)vp[2], 0.f);
    } else if (MODE == 1) {
        const ds X = ds_from_double(xp[0]), Y = ds_from_double(xp[1]), Z = ds_from_double(xp[2]);
        const ds VX = ds_from_double(vp[0]), VY = ds_from_double(vp[1]), VZ = ds_from_double(vp[2]);
        const ds M = ds_from_double(m);
        js.q0[i] = make_float4(X.hi, Y.hi, Z.hi, M.hi);
        js.q1[i] = make_float4(X.lo, Y.lo, Z.lo, M.lo);
        js.q2[i] = make_float4(VX.hi, VY.hi, VZ.hi, 0.f);
        js.q3[i] = make_float4(VX.lo, VY.lo, VZ.lo, 0.f);
    } else {
        js.px[i] = xp[0]; js.py[i] = xp[1]; js.pz[i] = xp[2]; js.pm[i] = m;
        js.vx[i] = vp[0]; js.vy[i] = vp[1]; js.vz[i] = vp[2];
    }
}

template <int MODE>
__global__ void __launch_bounds__(WG) predict_kernel(StateView s, JStreamView js,
                                                     const int64_t *t_ptr, const DevControl *ctl,
                                                     int32_t guard) {
    if (guard && ctl->n_act == 0) return;
    const int64_t t = t_ptr ? *t_ptr : ctl->t_next;
    for (int32_t i = blockIdx.x * WG + threadIdx.x; i < s.n; i += gridDim.x * WG)
        predict_store<MODE>(s, js, i, t);
}

// ------------------------------------------------------------------------------------------
// Sec. 2 Eq. initTimestep and power-of-two rounding; and the start-of-run state.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ int32_t level_from_dt(double dt, int32_t lmin, int32_t lmax) {
    int32_t l = lmin;
    while (l < lmax && __builtin_ldexp(1.0, -l) > dt) ++l;
    return l;
}

__global__ void __launch_bounds__(WG) zero_ticks(int64_t *tick, int32_t n) {
    for (int32_t i = blockIdx.x * WG + threadIdx.x; i < n; i += gridDim.x * WG) tick[i] = 0;
}

// Zero two small word arrays (a fill kernel, so that the call stays capturable in a graph).
__global__ void __launch_bounds__(WG) zero_words(int64_t *a, int32_t na, int32_t *b, int32_t nb) {
    for (int32_t i = threadIdx.x; i < na; i += WG) a[i] = 0;
    for (int32_t i = threadIdx.x; i < nb; i += WG) b[i] = 0;
}

__global__ void __launch_bounds__(WG) reset_control(DevControl *ctl) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl->t_cur = 0; ctl->t_next = 0; ctl->t_end = INT64_MAX; ctl->n_steps = 0;
        ctl->n_active_sum = 0; ctl->n_act = 0; ctl->flags = 0; ctl->t_cand = 0;
        ctl->n_pending = 0; ctl->done = 0; ctl->flag_nonfinite = 0; ctl->flag_dtmin = 0;
        ctl->flag_sched = 0; ctl->sel = 0;
    }
}

__global__ void __launch_bounds__(WG) set_t_end(DevControl *ctl, int64_t t_end) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl->t_end = t_end;
        ctl->done = 0;
    }
}

struct StateRW {
    double *x, *v, *a, *k, *m, *pot;
    int64_t *tick;
    int32_t *level;
    int32_t n;
    double tick_len;
};

__global__ void __launch_bounds__(WG) init_levels(StateRW s, const double *acc, const double *jerk,
                                                  const double *pot, double eta, int32_t lmin,
                                                  int32_t lmax, DevControl *ctl) {
    const int32_t n = s.n;
    for (int32_t i = blockIdx.x * WG + threadIdx.x; i < n; i += gridDim.x * WG) {
        double na = 0.0, nk = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double a = acc[c * (int64_t)n + i], k = jerk[c * (int64_t)n + i];
            s.a[c * (int64_t)n + i] = a;
            s.k[c * (int64_t)n + i] = k;
            na = __builtin_fma(a, a, na);
            nk = __builtin_fma(k, k, nk);
        }
        s.pot[i] = pot[i];
        na = __builtin_sqrt(na);
        nk = __builtin_sqrt(nk);
        const double dt = nk > 0.0 ? eta * na / nk : __builtin_inf();
        if (!__builtin_isfinite(na) || !__builtin_isfinite(nk)) ctl->flag_nonfinite = 1;
        s.level[i] = level_from_dt(dt, lmin, lmax);
        s.tick[i] = 0;
    }
}

// ------------------------------------------------------------------------------------------
// Sec. 2 corrector (FP64) on the selected block.
// ------------------------------------------------------------------------------------------
// Corrector of particle i over its step dt from the new acceleration/jerk/potential; writes
// the corrected state, the criterion inputs and the particle's time; false if not finite.
__device__ __forceinline__ bool correct_particle(const StateRW &s, int32_t i, double dt,
                                                 const double a1v[3], const double k1v[3],
                                                 double pot1, int64_t t_new, double *crit,
                                                 double *crit_num = nullptr,
                                                 double *crit_den = nullptr) {
    const int32_t n = s.n;
    const double idt = 1.0 / dt;  // a power of two: exact
    const double dt2 = dt * dt, dt3 = dt2 * dt, dt4 = dt3 * dt, dt5 = dt4 * dt;
    double na1 = 0.0, nk1 = 0.0, na2p = 0.0, na3 = 0.0;
    bool ok = true;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int64_t e = c * (int64_t)n + i;
        const double x = s.x[e], v = s.v[e], a0 = s.a[e], k0 = s.k[e];
        const double a1 = a1v[c], k1 = k1v[c];
        double xp, vp;
        predict_one(dt, x, v, a0, k0, xp, vp);
        const double da = a0 - a1;
        const double a2 = (-6.0 * da * idt - (4.0 * k0 + 2.0 * k1)) * idt;
        const double a3 = (12.0 * da * idt + 6.0 * (k0 + k1)) * idt * idt;
        const double xn = xp + a2 * (dt4 * (1.0 / 24.0)) + a3 * (dt5 * (1.0 / 120.0));
        const double vn = vp + a2 * (dt3 * (1.0 / 6.0)) + a3 * (dt4 * (1.0 / 24.0));
        const double a2p = a2 + a3 * dt;
        ok = ok && __builtin_isfinite(xn) && __builtin_isfinite(vn) && __builtin_isfinite(a2p);
        s.x[e] = xn; s.v[e] = vn; s.a[e] = a1; s.k[e] = k1;
        na1 = __builtin_fma(a1, a1, na1);
        nk1 = __builtin_fma(k1, k1, nk1);
        na2p = __builtin_fma(a2p, a2p, na2p);
        na3 = __builtin_fma(a3, a3, na3);
    }
    s.pot[i] = pot1;
    na1 = __builtin_sqrt(na1); nk1 = __builtin_sqrt(nk1);
    na2p = __builtin_sqrt(na2p); na3 = __builtin_sqrt(na3);
    const double num = na1 * na2p + nk1 * nk1, den = nk1 * na3 + na2p * na2p;
    if (crit) {
        crit[2 * (int64_t)i] = num;
        crit[2 * (int64_t)i + 1] = den;
    }
    if (crit_num) *crit_num = num;
    if (crit_den) *crit_den = den;
    s.tick[i] = t_new;
    return ok;
}

__global__ void __launch_bounds__(WG) correct_kernel(StateRW s, const int32_t *active,
                                                     const double *acc, const double *jerk,
                                                     const double *pot, int32_t ld,
                                                     double *crit, DevControl *ctl) {
    const int32_t n_act = ctl->n_act;
    const int64_t t_next = ctl->t_next;
    for (int32_t q = blockIdx.x * WG + threadIdx.x; q < n_act; q += gridDim.x * WG) {
        const int32_t i = active[q];
        const double dt = (double)(t_next - s.tick[i]) * s.tick_len;
        double a1[3], k1[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            a1[c] = acc[c * (int64_t)ld + q];
            k1[c] = jerk[c * (int64_t)ld + q];
        }
        if (!correct_particle(s, i, dt, a1, k1, pot[q], t_next, crit)) ctl->flag_nonfinite = 1;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && n_act > 0) {
        ctl->t_cur = t_next;
        ctl->n_steps += 1;
        ctl->n_active_sum += n_act;
        ctl->n_pending = n_act;
    }
}

// ------------------------------------------------------------------------------------------
// Sec. 2 block scheduling.
// ------------------------------------------------------------------------------------------
// Power-of-two rule for a particle on level l at tick t whose criterion gives dt: halve until
// not above dt; or double once when dt allows it, t is a multiple of the doubled step and the
// doubled step is within 2^-lmin.
__device__ __forceinline__ int32_t next_level(double dt, int32_t l, int64_t t, int32_t lmin,
                                              int32_t lmax) {
    if (dt < __builtin_ldexp(1.0, -l)) {
        while (l < lmax && __builtin_ldexp(1.0, -l) > dt) ++l;
    } else if (l > lmin && dt >= __builtin_ldexp(1.0, -(l - 1))) {
        const int64_t two_dt = (int64_t)1 << (lmax - l + 1);
        if (t % two_dt == 0) --l;
    }
    return l;
}

// New level of each particle corrected last (Eq. timestep, power-of-two rules).
__global__ void __launch_bounds__(WG) sched_newlevel(StateRW s, const int32_t *active,
                                                     const double *crit, double eta,
                                                     int32_t lmin, int32_t lmax,
                                                     DevControl *ctl) {
    const int32_t np = ctl->n_pending;
    for (int32_t q = blockIdx.x * WG + threadIdx.x; q < np; q += gridDim.x * WG) {
        const int32_t i = active[q];
        const double num = crit[2 * (int64_t)i], den = crit[2 * (int64_t)i + 1];
        const double dt = den > 0.0 ? __builtin_sqrt(eta * num / den) : __builtin_inf();
        if (__builtin_isnan(dt)) ctl->flag_nonfinite = 1;
        else if (dt < s.tick_len) ctl->flag_dtmin = 1;
        s.level[i] = next_level(dt, s.level[i], s.tick[i], lmin, lmax);
    }
}

__device__ __forceinline__ int64_t wg_min_i64(int64_t v, int64_t *red) {
    // wave minimum by shuffles, then across the 4 waves through LDS
    for (int off = 32; off > 0; off >>= 1) {
        const int64_t o = __shfl_xor(v, off, 64);
        v = o < v ? o : v;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    int64_t r = red[0];
    for (int w = 1; w < WG / 64; ++w) r = red[w] < r ? red[w] : r;
    return r;
}

__device__ __forceinline__ int64_t wg_sum_i64(int64_t v, int64_t *red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    int64_t r = 0;
    for (int w = 0; w < WG / 64; ++w) r += red[w];
    return r;
}

struct SchedView {
    const int64_t *tick;
    const int32_t *level;
    int32_t n, lmax, chunk, groups;
    int64_t *wgmin;
    int32_t *cnt;
    int32_t *active;
};

// Pass 1: per-workgroup minimum of t_i + dt_i over its contiguous chunk.
__global__ void __launch_bounds__(WG) sched_min(SchedView v) {
    __shared__ int64_t red[WG / 64];
    const int32_t lo = blockIdx.x * v.chunk;
    const int32_t hi = lo + v.chunk < v.n ? lo + v.chunk : v.n;
    int64_t m = INT64_MAX;
    for (int32_t i = lo + threadIdx.x; i < hi; i += WG) {
        const int64_t tn = v.tick[i] + ((int64_t)1 << (v.lmax - v.level[i]));
        m = tn < m ? tn : m;
    }
    m = wg_min_i64(m, red);
    if (threadIdx.x == 0) v.wgmin[blockIdx.x] = m;
}

__device__ __forceinline__ int64_t global_min(const SchedView &v, int64_t *red) {
    int64_t m = INT64_MAX;
    for (int32_t g = threadIdx.x; g < v.groups; g += WG) m = v.wgmin[g] < m ? v.wgmin[g] : m;
    return wg_min_i64(m, red);
}

// Pass 2: the block time t_next = min over all, and each chunk's count of block members.
__global__ void __launch_bounds__(WG) sched_count(SchedView v, DevControl *ctl) {
    __shared__ int64_t red[WG / 64];
    const int64_t tc = global_min(v, red);
    const bool take = tc <= ctl->t_end;
    const int32_t lo = blockIdx.x * v.chunk;
    const int32_t hi = lo + v.chunk < v.n ? lo + v.chunk : v.n;
    int64_t c = 0;
    if (take)
        for (int32_t i = lo + threadIdx.x; i < hi; i += WG)
            c += (v.tick[i] + ((int64_t)1 << (v.lmax - v.level[i]))) == tc;
    c = wg_sum_i64(c, red);
    if (threadIdx.x == 0) {
        v.cnt[blockIdx.x] = (int32_t)c;
        if (blockIdx.x == 0) {
            ctl->t_cand = tc;
            ctl->done = take ? 0 : 1;
        }
    }
}

// Pass 3: ordered compaction of the block members into the active list (ascending index).
__global__ void __launch_bounds__(WG) sched_scatter(SchedView v, DevControl *ctl) {
    __shared__ int64_t red[WG / 64];
    __shared__ int32_t wsum[WG / 64];
    const int64_t tc = ctl->t_cand;
    const bool take = ctl->done == 0;
    // exclusive prefix of the chunk counts, and the total
    int64_t before = 0, total = 0;
    for (int32_t g = threadIdx.x; g < v.groups; g += WG) {
        before += g < (int32_t)blockIdx.x ? v.cnt[g] : 0;
        total += v.cnt[g];
    }
    before = wg_sum_i64(before, red);
    total = wg_sum_i64(total, red);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int32_t lo = blockIdx.x * v.chunk;
    const int32_t hi = lo + v.chunk < v.n ? lo + v.chunk : v.n;
    int32_t base = (int32_t)before;
    if (take) {
        for (int32_t i0 = lo; i0 < hi; i0 += WG) {
            const int32_t i = i0 + threadIdx.x;
            const bool f = i < hi && (v.tick[i] + ((int64_t)1 << (v.lmax - v.level[i]))) == tc;
            const uint64_t mask = __ballot(f);
            const int32_t below = __popcll(mask & ((1ull << lane) - 1ull));
            __syncthreads();
            if (lane == 0) wsum[wave] = __popcll(mask);
            __syncthreads();
            int32_t off = base;
            for (int w = 0; w < wave; ++w) off += wsum[w];
            if (f) v.active[off + below] = i;
            for (int w = 0; w < WG / 64; ++w) base += wsum[w];
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl->n_act = take ? (int32_t)total : 0;
        if (take) ctl->t_next = tc;
        ctl->n_pending = 0;
    }
}

// ------------------------------------------------------------------------------------------
// Fused block step (Sec. 2), the launch sequence of the composite step call: select + predict,
// force, then the reduction with the corrector and the new levels.  Particles on one
// level share their time: the power-of-two rules keep each t_i a multiple of dt_i and every
// particle is corrected at every multiple of its step, so t_i is the last multiple of dt_i not
// after the current time.  The next block time is therefore the first multiple of the finest
// occupied step after the current time, and the block is every particle with t_i + dt_i equal
// to it.  A per-level histogram in the control record gives the finest level without a pass
// over all particles, so one pass both counts the block members of each chunk and predicts
// every particle; the corrector assigns the new levels at once and posts the level changes to
// the histogram.
// ------------------------------------------------------------------------------------------
constexpr int NLEV = 64;   // levels 0 .. lmax <= 52

__global__ void __launch_bounds__(WG) hist_clear(DevControl *ctl) {
    if (blockIdx.x == 0 && threadIdx.x < NLEV) ctl->hist[threadIdx.x] = 0;
}

__global__ void __launch_bounds__(WG) hist_build(const int32_t *level, int32_t n, DevControl *ctl) {
    __shared__ int32_t h[NLEV];
    if (threadIdx.x < NLEV) h[threadIdx.x] = 0;
    __syncthreads();
    for (int32_t i = blockIdx.x * WG + threadIdx.x; i < n; i += gridDim.x * WG)
        atomicAdd(&h[level[i] & (NLEV - 1)], 1);
    __syncthreads();
    if (threadIdx.x < NLEV && h[threadIdx.x] != 0) atomicAdd(&ctl->hist[threadIdx.x], h[threadIdx.x]);
}

// One workgroup per chunk of v.chunk consecutive particles: the block time from the histogram,
// the prediction of every particle, and the chunk's block members appended to the block list.
// The chunk reserves its slots with one 64-bit atomic add on the control record (its member
// count to the low word, one finished chunk to the high word); the chunk whose add completes
// the high word knows the block size and writes the block record, then clears the word for the
// next step.  Members are in ascending order within a chunk and chunks in the order their adds
// land: a member's force and corrector do not depend on its place in the list (every row is
// summed alone, in an order set by the block size), so the states are those of the ordered
// list the separate calls build.
template <int MODE>
__global__ void __launch_bounds__(WG) fused_select_predict(SchedView v, StateView s,
                                                           JStreamView js, DevControl *ctl) {
    __shared__ int64_t red[WG / 64];
    __shared__ int32_t wsum[WG / 64];
    __shared__ int32_t sbase;
    int32_t lfine = -1;
    for (int32_t l = v.lmax; l >= 0; --l)
        if (ctl->hist[l] > 0) {
            lfine = l;
            break;
        }
    const int64_t dtf = lfine >= 0 ? (int64_t)1 << (v.lmax - lfine) : 1;
    const int64_t t_next = (ctl->t_cur / dtf + 1) * dtf;
    const bool take = lfine >= 0 && t_next <= ctl->t_end;
    const int32_t lo = blockIdx.x * v.chunk;
    const int32_t hi = lo + v.chunk < v.n ? lo + v.chunk : v.n;
    int64_t c = 0;
    if (take) {
        for (int32_t i = lo + threadIdx.x; i < hi; i += WG) {
            const int64_t tn = v.tick[i] + ((int64_t)1 << (v.lmax - v.level[i]));
            if (tn < t_next) ctl->flag_sched = 1;
            c += tn == t_next;
            predict_store<MODE>(s, js, i, t_next);
        }
    }
    c = wg_sum_i64(c, red);  // equal on every work-item
    if (threadIdx.x == 0) {
        const uint64_t old = atomicAdd((unsigned long long *)&ctl->sel,
                                       (unsigned long long)((1ull << 32) | (uint64_t)c));
        sbase = (int32_t)(old & 0xffffffffull);
        if ((int32_t)(old >> 32) == v.groups - 1) {  // every other chunk has added
            ctl->n_act = take ? sbase + (int32_t)c : 0;
            if (take) ctl->t_next = t_next;
            ctl->t_cand = t_next;
            ctl->done = take ? 0 : 1;
            ctl->n_pending = 0;
            atomicExch((unsigned long long *)&ctl->sel, 0ull);
        }
    }
    __syncthreads();
    if (c == 0) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int32_t base = sbase;
    for (int32_t i0 = lo; i0 < hi; i0 += WG) {
        const int32_t i = i0 + threadIdx.x;
        const bool f = i < hi && (v.tick[i] + ((int64_t)1 << (v.lmax - v.level[i]))) == t_next;
        const uint64_t mask = __ballot(f);
        const int32_t below = __popcll(mask & ((1ull << lane) - 1ull));
        __syncthreads();
        if (lane == 0) wsum[wave] = __popcll(mask);
        __syncthreads();
        int32_t off = base;
        for (int w = 0; w < wave; ++w) off += wsum[w];
        if (f) v.active[off + below] = i;
        for (int w = 0; w < WG / 64; ++w) base += wsum[w];
    }
}

// The block step's second pass and corrector in one launch: for each block row the
// fixed-order sum of its K partial planes, exactly as force_reduce forms it (wave w of RW adds
// the planes k = w mod RW into four running sums, the waves' totals added in wave order), then
// the corrector (Sec. 2) with the block particle's new level assigned at once (Eq. timestep,
// power-of-two rules) and the level change posted to the per-level histogram.  A unit is RC_ROWS consecutive block rows: lane c * RC_ROWS + r
// of every wave takes sum c of row r; wave 0 gathers the 7 sums of row r into lane r, which
// corrects it.  Units are dealt to the 8 XCDs in contiguous runs, so the halves of a 128-byte
// line of a partial plane are read on one XCD.  With K = 1 the force wrote the sums to
// acc/jerk/pot directly and only the corrector runs.
constexpr int RC_ROWS = 8;

template <bool FIXED>
__global__ void __launch_bounds__(WG_REDUCE) reduce_correct_level(ForceCommon fc, int32_t ib,
                                                                  StateRW s, double eta,
                                                                  int32_t lmin, int32_t lmax,
                                                                  DevControl *ctl) {
    __shared__ double part[RW][64];
    __shared__ int64_t ipart[FIXED ? RW : 1][64];
    __shared__ int32_t ibad[FIXED ? RW : 1][64];
    __shared__ int32_t dh[NLEV];
    __shared__ int32_t any;
    if (threadIdx.x < NLEV) dh[threadIdx.x] = 0;
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    const int32_t n_act = ctl->n_act < fc.n_i_max ? ctl->n_act : fc.n_i_max;
    const int64_t t_next = ctl->t_next;
    if (n_act <= 0) return;
    const ForcePlan pl = make_plan(n_act, fc.n, ib, fc.target, fc.kmax, fc.smax);
    const int32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int32_t c = lane / RC_ROWS, r = lane % RC_ROWS;  // c = 7: idle lanes
    const int32_t U = (n_act + RC_ROWS - 1) / RC_ROWS;
    const int32_t per = (int32_t)gridDim.x >> 3, x = blockIdx.x & 7, chunk = (U + 7) >> 3;
    const int32_t u_end = (x + 1) * chunk < U ? (x + 1) * chunk : U;
    for (int32_t u = x * chunk + (int32_t)(blockIdx.x >> 3); u < u_end; u += per) {
        const int32_t q = u * RC_ROWS + r;
        const bool live = c < 7 && q < n_act;
        double t = 0.0;
        if (pl.K == 1) {
            if (w == 0 && live)
                t = c < 3 ? fc.acc[c * (int64_t)fc.ld + q]
                  : c < 6 ? fc.jerk[(c - 3) * (int64_t)fc.ld + q] : fc.pot[q];
        } else {
            const double *src = fc.partial + (int64_t)(c < 7 ? c : 0) * pl.P + q;
            if constexpr (FIXED) {
                int64_t sum = 0;
                int32_t bad = 0;
                if (live) {
                    for (int32_t k = w; k < pl.K; k += RW) {
                        const int64_t v = (int64_t)__double_as_longlong(src[(int64_t)k * 7 * pl.P]);
                        bad |= v == INT64_MIN;
                        ModeF32Fixed::add(sum, v, bad);
                    }
                }
                ipart[w][lane] = sum;
                ibad[w][lane] = bad;
            } else {
                double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
                if (live) {
                    const int64_t st = (int64_t)RW * 7 * pl.P;
                    int32_t k = w;
                    for (; k + 3 * RW < pl.K; k += 4 * RW) {
                        const double *b = src + (int64_t)k * 7 * pl.P;
                        s0 += b[0]; s1 += b[st]; s2 += b[2 * st]; s3 += b[3 * st];
                    }
                    for (; k < pl.K; k += RW) s0 += src[(int64_t)k * 7 * pl.P];
                }
                part[w][lane] = ((s0 + s1) + s2) + s3;
            }
            __syncthreads();
            if (w == 0 && live) {
                if constexpr (FIXED) {
                    int64_t sum = ipart[0][lane];
                    int32_t bad = ibad[0][lane];
#pragma unroll
                    for (int k = 1; k < RW; ++k) {
                        bad |= ibad[k][lane];
                        ModeF32Fixed::add(sum, ipart[k][lane], bad);
                    }
                    const int F = c < 3 ? ModeF32Fixed::F_ACC : c < 6 ? ModeF32Fixed::F_JERK
                                                                      : ModeF32Fixed::F_POT;
                    t = bad ? __builtin_nan("") : __builtin_ldexp((double)sum, -F);
                    if (c == 6) t = -t;
                } else {
                    t = part[0][lane];
#pragma unroll
                    for (int k = 1; k < RW; ++k) t += part[k][lane];
                }
            }
        }
        if (w == 0) {
            if (live && !__builtin_isfinite(t)) ctl->flag_nonfinite = 1;
            double v[7];
#pragma unroll
            for (int k = 0; k < 7; ++k) v[k] = __shfl(t, k * RC_ROWS + r, 64);
            if (lane < RC_ROWS && q < n_act) {
                const int32_t i = fc.ilist[q];
                const double dt = (double)(t_next - s.tick[i]) * s.tick_len;
                const double a1[3] = {v[0], v[1], v[2]}, k1[3] = {v[3], v[4], v[5]};
                double num, den;
                if (!correct_particle(s, i, dt, a1, k1, v[6], t_next, nullptr, &num, &den))
                    ctl->flag_nonfinite = 1;
                const double dtn = den > 0.0 ? __builtin_sqrt(eta * num / den) : __builtin_inf();
                if (__builtin_isnan(dtn)) ctl->flag_nonfinite = 1;
                else if (dtn < s.tick_len) ctl->flag_dtmin = 1;
                const int32_t l0 = s.level[i];
                const int32_t l1 = next_level(dtn, l0, t_next, lmin, lmax);
                if (l1 != l0) {
                    s.level[i] = l1;
                    atomicAdd(&dh[l0 & (NLEV - 1)], -1);
                    atomicAdd(&dh[l1 & (NLEV - 1)], 1);
                    any = 1;
                }
            }
        }
        __syncthreads();  // part and ipart are written again by the next unit
    }
    __syncthreads();
    if (any && threadIdx.x < NLEV && dh[threadIdx.x] != 0)
        atomicAdd(&ctl->hist[threadIdx.x], dh[threadIdx.x]);
    if (blockIdx.x == 0 && threadIdx.x == 0) {  // nothing in this launch reads these
        ctl->t_cur = t_next;
        ctl->n_steps += 1;
        ctl->n_active_sum += n_act;
        ctl->n_pending = 0;
    }
}

// ------------------------------------------------------------------------------------------
// Calibration: the FP32 fused multiply-add issue rate (not part of the method).  Every
// work-item runs FMA_CHAINS independent chains acc += x_c * m for `iters` iterations (two-operand
// v_fmac_f32, no packed FP32), so the rate is bounded by VALU issue alone; the sums are stored
// only if they hit an impossible value, which keeps the work from being removed.
// ------------------------------------------------------------------------------------------
constexpr int FMA_CHAINS = 16;

// VOPND: the multiplier is a vector register (m + dm * lane, dm = 0 at launch) instead of a
// scalar operand.
template <bool VOPND>
__global__ void __launch_bounds__(WG) fma_probe(int32_t iters, float m, float dm, float *sink) {
    float x[FMA_CHAINS], acc[FMA_CHAINS];
#pragma unroll
    for (int c = 0; c < FMA_CHAINS; ++c) {
        x[c] = (float)(threadIdx.x + c) * 1e-3f;
        acc[c] = (float)c;
    }
    const float mv = VOPND ? m + dm * (float)threadIdx.x : m;
    for (int32_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < FMA_CHAINS; ++c) acc[c] = __builtin_fmaf(x[c], mv, acc[c]);
    }
    float t = 0.0f;
#pragma unroll
    for (int c = 0; c < FMA_CHAINS; ++c) t += acc[c];
    if (t == -1.0f) sink[0] = t;
}

// ------------------------------------------------------------------------------------------
// Sec. 4.2 energy diagnostic (FP64).
// ------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(WG) energy_predict(StateView s, const DevControl *ctl,
                                                     double *xp, double *vp) {
    const int32_t n = s.n;
    const int64_t t = ctl->t_cur;
    for (int32_t i = blockIdx.x * WG + threadIdx.x; i < n; i += gridDim.x * WG) {
        const double D = (double)(t - s.tick[i]) * s.tick_len;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int64_t e = c * (int64_t)n + i;
            predict_one(D, s.x[e], s.v[e], s.a[e], s.k[e], xp[e], vp[e]);
        }
    }
}

// Per particle: m_i sum_{j != i} m_j s^(-1/2) (tile sums folded with Neumaier compensation)
// and m_i |v_i|^2 / 2.
__global__ void __launch_bounds__(WG) energy_pairs(const double *xp, const double *vp,
                                                   const double *m, int32_t n, double eps2,
                                                   double *w_out, double *k_out) {
    __shared__ double sx[TJ], sy[TJ], sz[TJ], sm[TJ];
    const int32_t ntiles = (n + TJ - 1) / TJ;
    for (int32_t ib = blockIdx.x; ib * WG < n; ib += gridDim.x) {
        const int32_t i = ib * WG + threadIdx.x;
        const int32_t ic = i < n ? i : 0;
        const double xi = xp[ic], yi = xp[(int64_t)n + ic], zi = xp[2 * (int64_t)n + ic];
        double s = 0.0, comp = 0.0;
        for (int32_t t = 0; t < ntiles; ++t) {
            __syncthreads();
            const int32_t j = t * TJ + threadIdx.x;
            sx[threadIdx.x] = j < n ? xp[j] : 0.0;
            sy[threadIdx.x] = j < n ? xp[(int64_t)n + j] : 0.0;
            sz[threadIdx.x] = j < n ? xp[2 * (int64_t)n + j] : 0.0;
            sm[threadIdx.x] = j < n ? m[j] : 0.0;
            __syncthreads();
            double ts = 0.0;
            for (int jj = 0; jj < TJ; ++jj) {
                const double dx = sx[jj] - xi, dy = sy[jj] - yi, dz = sz[jj] - zi;
                const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, __builtin_fma(dx, dx, eps2)));
                const double term = sm[jj] * rsqrt_f64(r2);
                ts += (t * TJ + jj == i || !(r2 > 0.0)) ? 0.0 : term;
            }
            const double y = s + ts;  // Neumaier step
            comp += __builtin_fabs(s) >= __builtin_fabs(ts) ? (s - y) + ts : (ts - y) + s;
            s = y;
        }
        if (i < n) {
            const double mi = m[i];
            w_out[i] = mi * (s + comp);
            const double vx = vp[i], vy = vp[(int64_t)n + i], vz = vp[2 * (int64_t)n + i];
            k_out[i] = 0.5 * mi * __builtin_fma(vz, vz, __builtin_fma(vy, vy, vx * vx));
        }
    }
}

// One workgroup of 1024: fixed-order compensated sums of both arrays.
__global__ void __launch_bounds__(1024) energy_reduce(const double *w, const double *kin,
                                                      int32_t n, double *out) {
    __shared__ double sw[1024], sk[1024];
    double a = 0.0, ca = 0.0, b = 0.0, cb = 0.0;
    for (int32_t i = threadIdx.x; i < n; i += 1024) {
        double y = a + w[i];
        ca += __builtin_fabs(a) >= __builtin_fabs(w[i]) ? (a - y) + w[i] : (w[i] - y) + a;
        a = y;
        y = b + kin[i];
        cb += __builtin_fabs(b) >= __builtin_fabs(kin[i]) ? (b - y) + kin[i] : (kin[i] - y) + b;
        b = y;
    }
    sw[threadIdx.x] = a + ca;
    sk[threadIdx.x] = b + cb;
    __syncthreads();
    for (int s = 512; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sw[threadIdx.x] += sw[threadIdx.x + s];
            sk[threadIdx.x] += sk[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = sk[0];
        out[1] = -0.5 * sw[0];
    }
}

}  // namespace nbody
