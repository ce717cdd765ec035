// scheme.h -- per-cell arithmetic of the two problems, shared by every
// kernel (swept phases, Standard steps) and by the host cores' share of a
// heterogeneous advance, so that all results are bit-identical.  Compiled
// with -ffp-contract=off so each expression is evaluated exactly as written
// (no fused multiply-add); divisions and square roots are correctly rounded
// on both sides (IEEE on the host, the HIP expansions on the GPU).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace swept {

// Heat (App. A update equation), r = alpha dt / dx^2, dx = dy:
// T' = (T + r*((T_{i+1} - 2T) + T_{i-1})) + r*((T_{j+1} - 2T) + T_{j-1}).
template <typename T>
__host__ __device__ __forceinline__ T heat_update(T c, T xp, T xm, T yp, T ym, T r)
{
    const T two_c = c + c;
    const T dxx = (xp - two_c) + xm;
    const T dyy = (yp - two_c) + ym;
    return (c + r * dxx) + r * dyy;
}

// ---------------------------------------------------------------- Euler
// State q = (rho, m = rho u, n = rho v, E).  Equation of state (App. B):
// p = (gamma-1)(E - (m u + n v)/2).
template <typename T>
__host__ __device__ __forceinline__ T pressure(const T q[4], T gm1)
{
    const T u = q[1] / q[0];
    const T v = q[2] / q[0];
    const T ke = q[1] * u + q[2] * v;
    return gm1 * (q[3] - T(0.5) * ke);
}

// Physical flux along the axis whose momentum is q[A] (A = 1: F, A = 2: G,
// App. B) and the signal speed |u_A| + c, c = sqrt(gamma p / rho).
template <typename T, int A>
__host__ __device__ __forceinline__ void phys_flux(const T q[4], T gamma, T gm1, T f[4], T& speed)
{
    constexpr int Bc = (A == 1) ? 2 : 1;
    const T rho = q[0];
    const T ua = q[A] / rho;
    const T ub = q[Bc] / rho;
    const T ke = q[A] * ua + q[Bc] * ub;
    const T p = gm1 * (q[3] - T(0.5) * ke);
    f[0] = q[A];
    f[A] = q[A] * ua + p;
    f[Bc] = q[A] * ub;
    f[3] = (q[3] + p) * ua;
    const T c = sqrt(gamma * p / rho);
    speed = fabs(ua) + c;
}

template <typename T>
__host__ __device__ __forceinline__ bool ratio_ok(T r)
{
    return r > T(0) && r < T(INFINITY);
}

// Scheme variant bits (the readings of the limiter and of the spectral
// radius, App. B): 0 = pressure-ratio minmod and Rusanov speed.
constexpr int kLimiterLiteral = 1;  // the limiter factors with the printed exponents
constexpr int kSpeedRoe = 2;        // spectral radius at the Roe-averaged state

// Roe-averaged signal speed |u~_A| + c~ of the face states L and R along
// axis A: sqrt(rho)-weighted velocities and total enthalpy H = (E + p)/rho,
// c~^2 = (gamma - 1)(H~ - (u~^2 + v~^2)/2).
template <typename T, int A>
__host__ __device__ __forceinline__ T roe_speed(const T L[4], const T R[4], T gm1)
{
    constexpr int Bc = (A == 1) ? 2 : 1;
    const T wl = sqrt(L[0]), wr = sqrt(R[0]);
    const T ual = L[A] / L[0], ubl = L[Bc] / L[0];
    const T uar = R[A] / R[0], ubr = R[Bc] / R[0];
    const T pl = gm1 * (L[3] - T(0.5) * (L[A] * ual + L[Bc] * ubl));
    const T pr = gm1 * (R[3] - T(0.5) * (R[A] * uar + R[Bc] * ubr));
    const T hl = (L[3] + pl) / L[0], hr = (R[3] + pr) / R[0];
    const T den = wl + wr;
    const T ua = (wl * ual + wr * uar) / den;
    const T ub = (wl * ubl + wr * ubr) / den;
    const T hh = (wl * hl + wr * hr) / den;
    const T c2 = gm1 * (hh - T(0.5) * (ua * ua + ub * ub));
    return fabs(ua) + sqrt(c2);
}

// Numerical flux through the face between cells b and c of the run
// a, b, c, d along axis A, given the four cell pressures (App. B):
// pressure-ratio reconstruction shared by the four variables, then the
// Rusanov form (F(Q_R) + F(Q_L) + s (Q_L - Q_R)) / 2.  V = 0: minmod face
// factors min(1/r_b, 1)/2 and min(r_c, 1)/2 and s = max(|u_L| + c_L,
// |u_R| + c_R); kLimiterLiteral swaps the factors to min(r_b, 1)/2 and
// min(1/r_c, 1)/2; kSpeedRoe takes s at the Roe-averaged state.
template <typename T, int A, int V = 0>
__host__ __device__ __forceinline__ void face_flux(const T qa[4], const T qb[4], const T qc[4], const T qd[4], T pa, T pb,
                                          T pc, T pd, T gamma, T out[4])
{
    const T gm1 = gamma - T(1);
    const T rb = (pc - pb) / (pb - pa);  // ratio at the left cell
    const T rc = (pd - pc) / (pc - pb);  // ratio at the right cell
    constexpr bool lit = (V & kLimiterLiteral) != 0;
    T L[4], R[4];
    if (ratio_ok(rb)) {
        const T f = lit ? rb : T(1) / rb;
        const T phi = T(0.5) * (f < T(1) ? f : T(1));
#pragma unroll
        for (int k = 0; k < 4; ++k) L[k] = qb[k] + phi * (qc[k] - qb[k]);
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) L[k] = qb[k];
    }
    if (ratio_ok(rc)) {
        const T f = lit ? T(1) / rc : rc;
        const T phi = T(0.5) * (f < T(1) ? f : T(1));
#pragma unroll
        for (int k = 0; k < 4; ++k) R[k] = qc[k] + phi * (qb[k] - qc[k]);
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) R[k] = qc[k];
    }
    T fL[4], fR[4], sL, sR;
    phys_flux<T, A>(L, gamma, gm1, fL, sL);
    phys_flux<T, A>(R, gamma, gm1, fR, sR);
    T s;
    if constexpr ((V & kSpeedRoe) != 0)
        s = roe_speed<T, A>(L, R, gm1);
    else
        s = sL > sR ? sL : sR;
#pragma unroll
    for (int k = 0; k < 4; ++k) out[k] = T(0.5) * ((fR[k] + fL[k]) + s * (L[k] - R[k]));
}

}  // namespace swept
