// adjoint.hpp -- gfx950 device code for differentiating shared-step Hermite runs.
//
// One shared step of the Sec. 2 scheme with fixed dt, written out as a map of the state
// (x, v, a, k) and the new force (a1, k1) = F(x_p, v_p, m) at the predicted state:
//   x_p = x + dt v + dt^2/2 a + dt^3/6 k,         v_p = v + dt a + dt^2/2 k,
//   x'  = x + dt v + 7/20 dt^2 a + 3/20 dt^2 a1 + 1/20 dt^3 k - 1/30 dt^3 k1,
//   v'  = v + dt/2 (a + a1) + dt^2/12 (k - k1),    a' = a1,  k' = k1
// (the corrector's a2 dt^4/24 + a3 dt^5/120 and a2 dt^3/6 + a3 dt^4/24 expanded).  Its
// vector-Jacobian product is the transposed linear part plus the VJP of F, whose pair form is
//   phi(d, u; A, B) = A.d s^-3/2 + B.u s^-3/2 - 3 (d.u)(B.d) s^-5/2
// (A, B: adjoints of the acceleration and jerk of i; d = x_j - x_i, u = v_j - v_i), with
//   dphi/dd = A s^-3/2 - 3 s^-5/2 [(A.d + B.u) d + (B.d) u + (d.u) B] + 15 s^-7/2 (d.u)(B.d) d
//   dphi/du = B s^-3/2 - 3 s^-5/2 (B.d) d,      dphi/dm_j = phi / m_j.
// Every particle p gathers, over all q != p, its i-side terms (A_p, B_p against q) and its
// j-side terms (A_q, B_q of q against p).
#pragma once

#include <type_traits>

#include "kernels.hpp"

namespace nbody {

// Predictor of every particle over the shared step dt, into the j-particle stream.
template <int MODE>
__global__ void __launch_bounds__(WG) shared_predict(StateView s, JStreamView js, double dt) {
    const int32_t n = s.n;
    for (int32_t i = blockIdx.x * WG + threadIdx.x; i < n; i += gridDim.x * WG) {
        double xp[3], vp[3];
#pragma unroll
        for (int c = 0; c < 3; ++c)
            predict_one(dt, s.x[c * (int64_t)n + i], s.v[c * (int64_t)n + i],
                        s.a[c * (int64_t)n + i], s.k[c * (int64_t)n + i], xp[c], vp[c]);
        const double m = s.m[i];
        if (MODE == 0) {
            js.px[i] = xp[0]; js.py[i] = xp[1]; js.pz[i] = xp[2];
            js.vm[i] = make_float4((float)vp[0], (float)vp[1], (float)vp[2], (float)m);
        } else {
            js.px[i] = xp[0]; js.py[i] = xp[1]; js.pz[i] = xp[2]; js.pm[i] = m;
            js.vx[i] = vp[0]; js.vy[i] = vp[1]; js.vz[i] = vp[2];
        }
    }
}

// Corrector of every particle over the shared step dt (advances each time by dt_ticks).
__global__ void __launch_bounds__(WG) shared_correct(StateRW s, const double *acc,
                                                     const double *jerk, const double *pot,
                                                     double dt, int64_t dt_ticks,
                                                     int32_t *flag) {
    const int32_t n = s.n;
    for (int32_t i = blockIdx.x * WG + threadIdx.x; i < n; i += gridDim.x * WG) {
        double a1[3], k1[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            a1[c] = acc[c * (int64_t)n + i];
            k1[c] = jerk[c * (int64_t)n + i];
        }
        if (!correct_particle(s, i, dt, a1, k1, pot[i], s.tick[i] + dt_ticks, nullptr)) *flag = 1;
    }
}

// Step VJP, first part: adjoints of the new force from those of the step's outputs.
//   a1_bar = 3/20 dt^2 x'_bar + dt/2 v'_bar + a'_bar,  k1_bar = -1/30 dt^3 x'_bar - dt^2/12 v'_bar + k'_bar
__global__ void __launch_bounds__(WG) vjp_pre(int32_t n, double dt, const double *xb,
                                              const double *vb, const double *ab,
                                              const double *kb, double *a1b, double *k1b) {
    const double dt2 = dt * dt, dt3 = dt2 * dt;
    for (int64_t e = blockIdx.x * (int64_t)WG + threadIdx.x; e < 3 * (int64_t)n;
         e += (int64_t)gridDim.x * WG) {
        a1b[e] = (3.0 / 20.0) * dt2 * xb[e] + 0.5 * dt * vb[e] + ab[e];
        k1b[e] = -(1.0 / 30.0) * dt3 * xb[e] - (1.0 / 12.0) * dt2 * vb[e] + kb[e];
    }
}

// Step VJP, last part: adjoints of the step's inputs, in place, from those of its outputs and
// of the predicted state (xpb, vpb: the force VJP).
__global__ void __launch_bounds__(WG) vjp_post(int32_t n, double dt, double *xb, double *vb,
                                               double *ab, double *kb, const double *xpb,
                                               const double *vpb) {
    const double dt2 = dt * dt, dt3 = dt2 * dt;
    for (int64_t e = blockIdx.x * (int64_t)WG + threadIdx.x; e < 3 * (int64_t)n;
         e += (int64_t)gridDim.x * WG) {
        const double X = xb[e], V = vb[e], XP = xpb[e], VP = vpb[e];
        xb[e] = X + XP;
        vb[e] = dt * X + V + dt * XP + VP;
        ab[e] = (7.0 / 20.0) * dt2 * X + 0.5 * dt * V + 0.5 * dt2 * XP + dt * VP;
        kb[e] = (1.0 / 20.0) * dt3 * X + (1.0 / 12.0) * dt2 * V + (1.0 / 6.0) * dt3 * XP +
                0.5 * dt2 * VP;
    }
}

template <class T> __device__ __forceinline__ T fma_t(T a, T b, T c);
template <> __device__ __forceinline__ float fma_t<float>(float a, float b, float c) {
    return __builtin_fmaf(a, b, c);
}
template <> __device__ __forceinline__ double fma_t<double>(double a, double b, double c) {
    return __builtin_fma(a, b, c);
}

// Pair terms of the force VJP for particle p against q, arithmetic type T.  d = x_q - x_p,
// u = v_q - v_p; (A, B) adjoints of p, (Aq, Bq) adjoints of q; rinv = s^-1/2 or 0 (self).
// With r3 = rinv^3, r5, r7 and du = d.u, the derivative of m_q (A.a + B.k) with respect to d
// is m_q [A r3 + c1 d + c2 u + c3 B] and with respect to u is m_q [B r3 + c2 d], where
// c1 = -3 r5 (A.d + B.u) + 15 r7 du B.d, c2 = -3 r5 B.d, c3 = -3 r5 du (even in (d, u)).
// p gains the i-side term with -m_q and its own (A, B), and the j-side term with +m_p and
// q's (Aq, Bq); both are added at once, the shared factors formed once:
//   gx += r3 (m_p Aq - m_q A) + (m_p c1q - m_q c1) d + (m_p c2q - m_q c2) u + c3 (m_p Bq - m_q B)
//   gu += r3 (m_p Bq - m_q B) + (m_p c2q - m_q c2) d
// and gm gains phi at (-d, -u) with q's adjoints: -(Aq.d + Bq.u) r3 - c3 Bq.d.
// p's adjoints come in negated (nA = -A, nB = -B) and the mass sum is kept negated (ngm = -gm):
// round-to-nearest is odd-symmetric, so every value is exactly the one the signs above give,
// and each product with a negated operand is a plain two-operand multiply or FMA rather than
// one carrying a negation modifier (which takes the slower three-operand encoding).
template <class T>
__device__ __forceinline__ void vjp_pair(T dx, T dy, T dz, T ux, T uy, T uz, T rinv, T mp, T mq,
                                         const T nA[3], const T nB[3], const T Aq[3],
                                         const T Bq[3], T gx[3], T gu[3], T &ngm) {
    const T r2 = rinv * rinv, r3 = rinv * r2, r5 = r3 * r2, r7 = r5 * r2;
    const T du = fma_t(dz, uz, fma_t(dy, uy, dx * ux));
    const T m3r5 = T(-3) * r5;
    const T c3 = m3r5 * du;
    const T f15 = (T(15) * r7) * du;
    const T nAd = fma_t(nA[2], dz, fma_t(nA[1], dy, nA[0] * dx));  // -A.d
    const T nBd = fma_t(nB[2], dz, fma_t(nB[1], dy, nB[0] * dx));  // -B.d
    const T nBu = fma_t(nB[2], uz, fma_t(nB[1], uy, nB[0] * ux));  // -B.u
    const T nc1 = fma_t(f15, nBd, m3r5 * (nAd + nBu));             // -c1
    const T nc2 = m3r5 * nBd;                                       // -c2
    const T Adq = fma_t(Aq[2], dz, fma_t(Aq[1], dy, Aq[0] * dx));
    const T Bdq = fma_t(Bq[2], dz, fma_t(Bq[1], dy, Bq[0] * dx));
    const T Buq = fma_t(Bq[2], uz, fma_t(Bq[1], uy, Bq[0] * ux));
    const T c1q = fma_t(f15, Bdq, m3r5 * (Adq + Buq));
    const T c2q = m3r5 * Bdq;
    const T C1 = fma_t(mp, c1q, mq * nc1);
    const T C2 = fma_t(mp, c2q, mq * nc2);
    const T d[3] = {dx, dy, dz}, u[3] = {ux, uy, uz};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const T Ab = fma_t(mp, Aq[k], mq * nA[k]);
        const T Bb = fma_t(mp, Bq[k], mq * nB[k]);
        gx[k] = fma_t(r3, Ab, fma_t(C1, d[k], fma_t(C2, u[k], fma_t(c3, Bb, gx[k]))));
        gu[k] = fma_t(r3, Bb, fma_t(C2, d[k], gu[k]));
    }
    ngm = fma_t(Adq + Buq, r3, fma_t(c3, Bdq, ngm));
}

struct VjpArgs {
    int32_t n;
    const double *px, *py, *pz;  // predicted positions (FP64)
    const float4 *vm;            // FP32 mode: predicted velocity + mass
    const double *pm, *vx, *vy, *vz;  // FP64 mode
    const double *ab, *kb;       // adjoints of acc and jerk, 3 x n
    double eps2;
    double *partial;             // [K][7][P]
    int32_t target, kmax;
};

template <class T>
struct VjpSmem {
    double x[TJ], y[TJ], z[TJ];
    T vx[TJ], vy[TJ], vz[TJ], m[TJ];
    T A[3][TJ], B[3][TJ];
};

// One staged tile of the force VJP for one particle p (position xp, velocity vp, mass mp,
// negated adjoints nA, nB).  SOFT (eps > 0): every separation is positive, and only a tile
// holding p's own slot (MASK, slot rel) needs a test, taken in a copy of the loop that masks
// that slot; without softening every pair at zero separation (the self pair among them) adds
// nothing.  Padding slots carry zero mass and zero adjoints and add exact zeros.
template <class T, bool SOFT, bool MASK>
__device__ __forceinline__ void vjp_tile(const VjpSmem<T> &sm, int32_t rel, double xp, double yp,
                                         double zp, T vxp, T vyp, T vzp, T mp, T eps2,
                                         const T nA[3], const T nB[3], T gx[3], T gu[3],
                                         T &ngm) {
#pragma unroll 1
    for (int jj = 0; jj < TJ; ++jj) {
        const T dx = (T)(sm.x[jj] - xp), dy = (T)(sm.y[jj] - yp), dz = (T)(sm.z[jj] - zp);
        const T ux = sm.vx[jj] - vxp, uy = sm.vy[jj] - vyp, uz = sm.vz[jj] - vzp;
        const T s = dx * dx + dy * dy + dz * dz + eps2;
        T rinv;
        if (std::is_same<T, float>::value) rinv = (T)__builtin_amdgcn_rsqf((float)s);
        else rinv = (T)rsqrt_f64((double)s);
        if (MASK && jj == rel) rinv = T(0);
        if (!SOFT && !(s > T(0))) rinv = T(0);
        const T Aq[3] = {sm.A[0][jj], sm.A[1][jj], sm.A[2][jj]};
        const T Bq[3] = {sm.B[0][jj], sm.B[1][jj], sm.B[2][jj]};
        vjp_pair<T>(dx, dy, dz, ux, uy, uz, rinv, mp, sm.m[jj], nA, nB, Aq, Bq, gx, gu, ngm);
    }
}

// Force VJP over all particles; j-split into K ranges, partial sums (7 per particle: x_bar,
// v_bar, m_bar) per range, summed by vjp_reduce.  MODE 0: float arithmetic on separations
// formed in double (tile sums folded into double); MODE 2: double throughout.  SOFT: eps > 0
// in the arithmetic type.
template <int MODE, bool SOFT>
__global__ void __launch_bounds__(WG) force_vjp_kernel(VjpArgs a) {
    using T = typename std::conditional<MODE == 0, float, double>::type;
    __shared__ VjpSmem<T> sm;
    const int32_t n = a.n;
    const ForcePlan pl = make_plan(n, n, WG, a.target, a.kmax);
    for (int32_t w = blockIdx.x; w < pl.items; w += gridDim.x) {
        const int32_t iblk = w / pl.K, ks = w - (w / pl.K) * pl.K;
        const int32_t p = iblk * WG + (int32_t)threadIdx.x;
        const int32_t pc = p < n ? p : 0;
        const int32_t own = p < n ? p : -1;  // p's own j-slot (none on padding lanes)
        const double xp = a.px[pc], yp = a.py[pc], zp = a.pz[pc];
        T vxp, vyp, vzp, mp;
        if (MODE == 0) {
            const float4 q = a.vm[pc];
            vxp = q.x; vyp = q.y; vzp = q.z; mp = q.w;
        } else {
            vxp = a.vx[pc]; vyp = a.vy[pc]; vzp = a.vz[pc]; mp = a.pm[pc];
        }
        T nA[3], nB[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            nA[k] = -(T)a.ab[k * (int64_t)n + pc];
            nB[k] = -(T)a.kb[k * (int64_t)n + pc];
            // opaque to the optimiser, which would otherwise fold the negation back into
            // modifiers on the products inside the pair loop
            asm volatile("" : "+v"(nA[k]), "+v"(nB[k]));
        }
        double S[7] = {0, 0, 0, 0, 0, 0, 0};
        const T eps2 = (T)a.eps2;
        const int32_t t0 = ks * pl.tps;
        const int32_t t1 = t0 + pl.tps < pl.ntiles ? t0 + pl.tps : pl.ntiles;
        for (int32_t t = t0; t < t1; ++t) {
            __syncthreads();
            {
                const int32_t j = t * TJ + (int32_t)threadIdx.x;
                const bool ok = j < n;
                const int32_t jc = ok ? j : 0;
                sm.x[threadIdx.x] = a.px[jc]; sm.y[threadIdx.x] = a.py[jc]; sm.z[threadIdx.x] = a.pz[jc];
                if (MODE == 0) {
                    const float4 q = a.vm[jc];
                    sm.vx[threadIdx.x] = q.x; sm.vy[threadIdx.x] = q.y; sm.vz[threadIdx.x] = q.z;
                    sm.m[threadIdx.x] = ok ? q.w : 0.f;
                } else {
                    sm.vx[threadIdx.x] = a.vx[jc]; sm.vy[threadIdx.x] = a.vy[jc];
                    sm.vz[threadIdx.x] = a.vz[jc]; sm.m[threadIdx.x] = ok ? a.pm[jc] : 0.0;
                }
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    sm.A[k][threadIdx.x] = ok ? (T)a.ab[k * (int64_t)n + jc] : T(0);
                    sm.B[k][threadIdx.x] = ok ? (T)a.kb[k * (int64_t)n + jc] : T(0);
                }
            }
            __syncthreads();
            T gx[3] = {0, 0, 0}, gu[3] = {0, 0, 0}, ngm = 0;
            const int32_t rel = own - t * TJ;
            // a tile holding some lane's own slot takes the masked loop (wave-uniform branch)
            if (SOFT && __ballot((uint32_t)rel < (uint32_t)TJ) != 0)
                vjp_tile<T, SOFT, true>(sm, rel, xp, yp, zp, vxp, vyp, vzp, mp, eps2, nA, nB, gx, gu, ngm);
            else
                vjp_tile<T, SOFT, false>(sm, rel, xp, yp, zp, vxp, vyp, vzp, mp, eps2, nA, nB, gx, gu, ngm);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                S[k] += (double)gx[k];
                S[3 + k] += (double)gu[k];
            }
            S[6] -= (double)ngm;
        }
        if (p < n) {
            double *base = a.partial + (int64_t)ks * 7 * pl.P + p;
#pragma unroll
            for (int k = 0; k < 7; ++k) base[(int64_t)k * pl.P] = S[k];
        }
    }
}

// Sums the K partial planes (fixed order): x_bar, v_bar of the predicted state written to
// (accumulate = 0) or added to (accumulate = 1) xpb, vpb; m_bar added to mb.
__global__ void __launch_bounds__(WG) vjp_reduce(int32_t n, const double *partial, int32_t target,
                                                 int32_t kmax, double *xpb, double *vpb,
                                                 double *mb, int32_t accumulate) {
    const ForcePlan pl = make_plan(n, n, WG, target, kmax);
    for (int32_t p = blockIdx.x * WG + threadIdx.x; p < n; p += gridDim.x * WG) {
        double o[7] = {0, 0, 0, 0, 0, 0, 0};
        for (int32_t k = 0; k < pl.K; ++k)
#pragma unroll
            for (int c = 0; c < 7; ++c) o[c] += partial[((int64_t)k * 7 + c) * pl.P + p];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int64_t e = c * (int64_t)n + p;
            xpb[e] = (accumulate ? xpb[e] : 0.0) + o[c];
            vpb[e] = (accumulate ? vpb[e] : 0.0) + o[3 + c];
        }
        mb[p] += o[6];
    }
}

}  // namespace nbody
