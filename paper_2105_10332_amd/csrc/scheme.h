// scheme.h -- per-cell arithmetic of the two problems, shared by every
// kernel (swept phases, Standard steps), so that Swept and Standard results
// are bit-identical.  Device code only; compiled with -ffp-contract=off so
// each expression is evaluated exactly as written (no fused multiply-add).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace swept {

// Heat (App. A update equation), r = alpha dt / dx^2, dx = dy:
// T' = (T + r*((T_{i+1} - 2T) + T_{i-1})) + r*((T_{j+1} - 2T) + T_{j-1}).
template <typename T>
__device__ __forceinline__ T heat_update(T c, T xp, T xm, T yp, T ym, T r)
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
__device__ __forceinline__ T pressure(const T q[4], T gm1)
{
    const T u = q[1] / q[0];
    const T v = q[2] / q[0];
    const T ke = q[1] * u + q[2] * v;
    return gm1 * (q[3] - T(0.5) * ke);
}

// Physical flux along the axis whose momentum is q[A] (A = 1: F, A = 2: G,
// App. B) and the signal speed |u_A| + c, c = sqrt(gamma p / rho).
template <typename T, int A>
__device__ __forceinline__ void phys_flux(const T q[4], T gamma, T gm1, T f[4], T& speed)
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
__device__ __forceinline__ bool ratio_ok(T r)
{
    return r > T(0) && r < T(INFINITY);
}

// Numerical flux through the face between cells b and c of the run
// a, b, c, d along axis A, given the four cell pressures (App. B):
// pressure-ratio minmod reconstruction shared by the four variables, then
// the Rusanov form (F(Q_R) + F(Q_L) + s (Q_L - Q_R)) / 2 with
// s = max(|u_L| + c_L, |u_R| + c_R).
template <typename T, int A>
__device__ __forceinline__ void face_flux(const T qa[4], const T qb[4], const T qc[4], const T qd[4], T pa, T pb,
                                          T pc, T pd, T gamma, T out[4])
{
    const T gm1 = gamma - T(1);
    const T rb = (pc - pb) / (pb - pa);  // ratio at the left cell
    const T rc = (pd - pc) / (pc - pb);  // ratio at the right cell
    T L[4], R[4];
    if (ratio_ok(rb)) {
        const T inv = T(1) / rb;
        const T phi = T(0.5) * (inv < T(1) ? inv : T(1));
#pragma unroll
        for (int k = 0; k < 4; ++k) L[k] = qb[k] + phi * (qc[k] - qb[k]);
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) L[k] = qb[k];
    }
    if (ratio_ok(rc)) {
        const T phi = T(0.5) * (rc < T(1) ? rc : T(1));
#pragma unroll
        for (int k = 0; k < 4; ++k) R[k] = qc[k] + phi * (qb[k] - qc[k]);
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) R[k] = qc[k];
    }
    T fL[4], fR[4], sL, sR;
    phys_flux<T, A>(L, gamma, gm1, fL, sL);
    phys_flux<T, A>(R, gamma, gm1, fR, sR);
    const T s = sL > sR ? sL : sR;
#pragma unroll
    for (int k = 0; k < 4; ++k) out[k] = T(0.5) * ((fR[k] + fL[k]) + s * (L[k] - R[k]));
}

}  // namespace swept
