/*
 * oracle.c -- plain CPU oracle for the two-dimensional swept rule
 * (Walker & Niemeyer, "The Two-Dimensional Swept Rule Applied on
 * Heterogeneous Architectures", arXiv:2105.10332).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only tests/, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header or constant with the HIP
 * library.
 *
 * What it computes.  The swept rule reaches exactly the result of the
 * one-step-at-a-time "Standard" solver (Sec. 3.1: both solvers share the
 * decomposition and the arithmetic; Sec. 3.3: every point is solved once).
 * The oracle is therefore M plain Standard steps, written as double loops
 * over the whole periodic grid:
 *   - heat:  forward-Euler, 3-point differences per axis (App. A, update
 *            equation), periodic unit square;
 *   - Euler: 2nd-order finite volume with a pressure-ratio minmod limiter,
 *            a Rusanov-form flux and explicit-midpoint RK2 (App. B);
 *   - the discrete adjoint of the heat run (reverse sweep of the transposed
 *     step, not in the paper) and the scalar diagnostics (CFL time step,
 *     conservation sums).
 *
 * The source is compiled twice: -DREAL=double -DSFX=_f64 and
 * -DREAL=float -DSFX=_f32.  Accumulations of scalar diagnostics are always
 * in double.  Build with -O2 -ffp-contract=off (no fused multiply-add, no
 * fast-math) so every expression is evaluated exactly as written.
 *
 * Layout: a field is N*N values, row-major, x fastest: index = j*N + i with
 * i the x (column) index and j the y (row) index; cell centres at
 * ((i+1/2)dx, (j+1/2)dy).  Euler state is four such planes in the order
 * rho, rho*u, rho*v, E.
 *
 * Readings of the paper taken here (the paper is garbled or silent):
 *   - heat update evaluated as (T + r*((T_{i+1}-2T)+T_{i-1})) + r*((T_{j+1}-2T)+T_{j-1})
 *     with 2T formed as T+T, r = alpha*dt/dx^2 (App. A, dx = dy);
 *   - Euler: conservation form Q_t + F_x + G_y = 0 with F, G as printed in
 *     App. B (the component equations printed above them have sign errors);
 *   - limiter: one pressure ratio r_i = (p_{i+1}-p_i)/(p_i-p_{i-1}) shared
 *     by all four variables; left face state Q_i + (min(1/r_i,1)/2)(Q_{i+1}-Q_i),
 *     right face state Q_{i+1} + (min(r_{i+1},1)/2)(Q_i-Q_{i+1}), each used
 *     only when its ratio lies in (0, +inf), otherwise the cell value
 *     (first order).  This is the textbook minmod MUSCL face value for the
 *     pressure itself; the printed exponents would anti-limit;
 *   - flux: F = (F(Q_R) + F(Q_L) + s (Q_L - Q_R)) / 2 with the spectral
 *     radius s = max(|u_L|+c_L, |u_R|+c_R), c = sqrt(gamma p / rho);
 *   - RK2: Q* = Q^n - (dt/2dx)(F_{i+1/2}-F_{i-1/2}) - (dt/2dy)(G_{j+1/2}-G_{j-1/2}),
 *     Q^{n+1} = Q^n - (dt/dx)(F*_{i+1/2}-F*_{i-1/2}) - (dt/dy)(G*...), the
 *     explicit midpoint rule (the printed signs and flux sums are garbled).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef REAL
#define REAL double
#endif
#ifndef SFX
#define SFX _f64
#endif
#define CAT2(a, b) a##b
#define CAT(a, b) CAT2(a, b)
#define NAME(f) CAT(f, SFX)

static inline int64_t wrap(int64_t i, int64_t n) { return (i % n + n) % n; }

/* ------------------------------------------------------------------ heat */

/* Boundaries: the paper's grid is periodic; it notes that other conditions
 * fit the same decomposition.  BC_DIRICHLET: every neighbour outside the
 * square is a ghost cell holding the fixed value bcv.  BC_NEUMANN (zero
 * flux): an outside neighbour holds the value of the edge cell itself. */
#define BC_PERIODIC 0
#define BC_DIRICHLET 1
#define BC_NEUMANN 2
#define BC_REFLECT 3 /* Euler slip wall, see euler_ghost */

/* Value of neighbour (i, j) of cell (ci, cj), which may lie outside the
 * square by one cell. */
static inline REAL neighbour(const REAL* T, int64_t N, int64_t i, int64_t j, int64_t ci, int64_t cj, int bc, REAL bcv)
{
    if (i >= 0 && i < N && j >= 0 && j < N) return T[j * N + i];
    if (bc == BC_DIRICHLET) return bcv;
    if (bc == BC_NEUMANN) return T[cj * N + ci];
    return T[wrap(j, N) * N + wrap(i, N)];
}

/* One forward-Euler step of the heat equation (App. A, update equation),
 * boundary bc (ghost value bcv for BC_DIRICHLET).  Tout may not alias Tin. */
void NAME(oracle_heat_step_bc)(const REAL* Tin, REAL* Tout, int64_t N, double r_in, int64_t bc, double bcv_in)
{
    const REAL r = (REAL)r_in, bcv = (REAL)bcv_in;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < N; ++j) {
        for (int64_t i = 0; i < N; ++i) {
            const REAL c = Tin[j * N + i];
            const REAL two_c = c + c;
            const REAL dxx = (neighbour(Tin, N, i + 1, j, i, j, (int)bc, bcv) - two_c) +
                             neighbour(Tin, N, i - 1, j, i, j, (int)bc, bcv);
            const REAL dyy = (neighbour(Tin, N, i, j + 1, i, j, (int)bc, bcv) - two_c) +
                             neighbour(Tin, N, i, j - 1, i, j, (int)bc, bcv);
            Tout[j * N + i] = (c + r * dxx) + r * dyy;
        }
    }
}

/* One periodic step. */
void NAME(oracle_heat_step)(const REAL* Tin, REAL* Tout, int64_t N, double r_in)
{
    NAME(oracle_heat_step_bc)(Tin, Tout, N, r_in, BC_PERIODIC, 0.0);
}

/* M heat steps with boundary bc.  T holds T^0 on entry and T^M on exit;
 * work is N*N scratch. */
void NAME(oracle_heat_run_bc)(REAL* T, REAL* work, int64_t N, double r, int64_t M, int64_t bc, double bcv)
{
    REAL* a = T;
    REAL* b = work;
    for (int64_t m = 0; m < M; ++m) {
        NAME(oracle_heat_step_bc)(a, b, N, r, bc, bcv);
        REAL* t = a; a = b; b = t;
    }
    if (a != T) memcpy(T, a, (size_t)(N * N) * sizeof(REAL));
}

/* M periodic heat steps. */
void NAME(oracle_heat_run)(REAL* T, REAL* work, int64_t N, double r, int64_t M)
{
    NAME(oracle_heat_run_bc)(T, work, N, r, M, BC_PERIODIC, 0.0);
}

/* Discrete 5-point Laplacian without the 1/dx^2 factor, L T, evaluated in
 * double: the quantity the diffusivity multiplies in the update. */
static double lap_at(const REAL* T, int64_t N, int64_t i, int64_t j)
{
    const double c = (double)T[j * N + i];
    return ((double)T[j * N + wrap(i + 1, N)] - 2.0 * c + (double)T[j * N + wrap(i - 1, N)]) +
           ((double)T[wrap(j + 1, N) * N + i] - 2.0 * c + (double)T[wrap(j - 1, N) * N + i]);
}

/* Discrete adjoint of M heat steps (not in the paper; the reverse sweep of
 * the forward recursion T^{m+1} = A T^m, A = I + r L).
 *   g     = dJ/dT^M on entry (N*N)
 *   gT0   = dJ/dT^0 on exit
 *   dJdr  = sum_{m=0}^{M-1} <lambda^{m+1}, L T^m>, lambda^m = A^T lambda^{m+1}
 * A is symmetric on the periodic grid (the neighbour relation is symmetric
 * and all four neighbour weights equal r), so A^T lambda is evaluated with
 * the same stencil as the forward step.  Every level T^0..T^{M-1} is kept
 * ((M+1)*N*N values in levels), which limits this to small cases. */
void NAME(oracle_heat_adjoint)(const REAL* T0, const REAL* g, REAL* gT0, double* dJdr,
                               int64_t N, double r, int64_t M, REAL* levels /* (M+1)*N*N */,
                               REAL* work /* N*N */)
{
    const int64_t NN = N * N;
    memcpy(levels, T0, (size_t)NN * sizeof(REAL));
    for (int64_t m = 0; m < M; ++m) NAME(oracle_heat_step)(levels + m * NN, levels + (m + 1) * NN, N, r);
    REAL* lam = gT0;
    memcpy(lam, g, (size_t)NN * sizeof(REAL));
    double acc = 0.0;
    for (int64_t m = M - 1; m >= 0; --m) {
        /* lam currently holds lambda^{m+1}; pair it with L T^m */
        const REAL* Tm = levels + m * NN;
        for (int64_t j = 0; j < N; ++j)
            for (int64_t i = 0; i < N; ++i) acc += (double)lam[j * N + i] * lap_at(Tm, N, i, j);
        NAME(oracle_heat_step)(lam, work, N, r); /* lambda^m = A^T lambda^{m+1} */
        memcpy(lam, work, (size_t)NN * sizeof(REAL));
    }
    *dJdr = acc;
}

/* L_bc T at cell (i, j) in double: the 5-point Laplacian (no 1/dx^2) with
 * the boundary's neighbour values (Dirichlet ghosts at bcv, zero flux, or
 * periodic), i.e. dT'/dr of the walled step T' = T + r L_bc T. */
static double lap_at_bc(const REAL* T, int64_t N, int64_t i, int64_t j, int bc, REAL bcv)
{
    const double c = (double)T[j * N + i];
    return ((double)neighbour(T, N, i + 1, j, i, j, bc, bcv) - 2.0 * c + (double)neighbour(T, N, i - 1, j, i, j, bc, bcv)) +
           ((double)neighbour(T, N, i, j + 1, i, j, bc, bcv) - 2.0 * c + (double)neighbour(T, N, i, j - 1, i, j, bc, bcv));
}

/* Discrete adjoint of M walled heat steps.  The walled step is affine,
 * T^{m+1} = A0 T^m + r b, with A0 = I + r L0 the step of the homogeneous
 * wall (Dirichlet ghosts at 0, or zero flux) and b the ghost terms
 * (bcv times the number of outside neighbours of a cell; 0 for zero flux).
 * L0 is symmetric for both walls, so lambda^m = A0^T lambda^{m+1} is the
 * homogeneous walled step applied to lambda, and
 * dJ/dr = sum_{m<M} <lambda^{m+1}, L_bc T^m> with L_bc the walled Laplacian
 * including the ghosts.  Arguments as oracle_heat_adjoint. */
void NAME(oracle_heat_adjoint_bc)(const REAL* T0, const REAL* g, REAL* gT0, double* dJdr, int64_t N, double r,
                                  int64_t M, REAL* levels, REAL* work, int64_t bc, double bcv_in)
{
    const int64_t NN = N * N;
    const REAL bcv = (REAL)bcv_in;
    memcpy(levels, T0, (size_t)NN * sizeof(REAL));
    for (int64_t m = 0; m < M; ++m)
        NAME(oracle_heat_step_bc)(levels + m * NN, levels + (m + 1) * NN, N, r, bc, bcv_in);
    REAL* lam = gT0;
    memcpy(lam, g, (size_t)NN * sizeof(REAL));
    double acc = 0.0;
    for (int64_t m = M - 1; m >= 0; --m) {
        const REAL* Tm = levels + m * NN;
        for (int64_t j = 0; j < N; ++j)
            for (int64_t i = 0; i < N; ++i) acc += (double)lam[j * N + i] * lap_at_bc(Tm, N, i, j, (int)bc, bcv);
        NAME(oracle_heat_step_bc)(lam, work, N, r, bc, 0.0); /* homogeneous wall: Dirichlet ghosts at 0 */
        memcpy(lam, work, (size_t)NN * sizeof(REAL));
    }
    *dJdr = acc;
}

/* J = 1/2 sum (T - Tstar)^2 in double. */
double NAME(oracle_l2_mismatch)(const REAL* T, const REAL* Tstar, int64_t n)
{
    double s = 0.0;
    for (int64_t k = 0; k < n; ++k) {
        const double d = (double)T[k] - (double)Tstar[k];
        s += d * d;
    }
    return 0.5 * s;
}

/* ----------------------------------------------------------------- Euler */

typedef struct { REAL v[4]; } state4;

static inline state4 load4(const REAL* Q, int64_t NN, int64_t k)
{
    state4 s;
    for (int c = 0; c < 4; ++c) s.v[c] = Q[c * NN + k];
    return s;
}

/* Equation of state (App. B): p = (gamma-1)(E - rho(u^2+v^2)/2), written
 * with the momenta and the velocities u = m/rho, v = n/rho:
 * p = (gamma-1)(E - (m u + n v)/2). */
static inline REAL pressure(state4 q, REAL gm1)
{
    const REAL u = q.v[1] / q.v[0];
    const REAL v = q.v[2] / q.v[0];
    const REAL ke = q.v[1] * u + q.v[2] * v;
    return gm1 * (q.v[3] - (REAL)0.5 * ke);
}

/* Flux in the direction whose momentum is component a (a=1: x, F; a=2:
 * y, G) and the other momentum is component b; also the signal speed
 * |u_a| + c.  F = (m_a, m_a u_a + p, m_a u_b, (E+p) u_a), u_a = m_a/rho,
 * c = sqrt(gamma p / rho). */
static inline void phys_flux(state4 q, int a, int b, REAL gamma, REAL gm1, REAL f[4], REAL* speed)
{
    const REAL rho = q.v[0];
    const REAL ua = q.v[a] / rho;
    const REAL ub = q.v[b] / rho;
    const REAL ke = q.v[a] * ua + q.v[b] * ub;
    const REAL p = gm1 * (q.v[3] - (REAL)0.5 * ke);
    f[0] = q.v[a];
    f[a] = q.v[a] * ua + p;
    f[b] = q.v[a] * ub;
    f[3] = (q.v[3] + p) * ua;
    const REAL c = (REAL)sqrt((double)(gamma * p / rho));
    *speed = (REAL)fabs((double)ua) + c;
}

static inline int ratio_ok(REAL r) { return r > (REAL)0 && r < (REAL)INFINITY; }

/* Scheme variants (App. B leaves two things open; the default is the
 * reading stated at the top of this file):
 *   SCHEME_LIMITER_LITERAL: the limiter factors with the exponents exactly
 *     as printed, min(r_i, 1)/2 for the left state and min(1/r_{i+1}, 1)/2
 *     for the right one (each still used only for a ratio in (0, inf));
 *   SCHEME_SPEED_ROE: the spectral radius of the flux Jacobian evaluated at
 *     the Roe-averaged state of the two face states, |u~| + c~, in place of
 *     the larger of the two one-sided speeds.  The bits combine. */
#define SCHEME_LIMITER_LITERAL 1
#define SCHEME_SPEED_ROE 2

/* Roe average of face states L and R for the direction whose momentum is
 * component a (other momentum b): weights sqrt(rho_L), sqrt(rho_R) applied
 * to u_a, u_b and the total enthalpy H = (E + p)/rho.  out = (u~_a, u~_b,
 * H~, |u~_a| + c~) with c~^2 = (gamma - 1)(H~ - (u~_a^2 + u~_b^2)/2); the
 * Roe matrix of the x-split Euler flux has eigenvalues u~_a - c~, u~_a
 * (twice) and u~_a + c~, so the last entry is its spectral radius. */
static void roe_average(state4 L, state4 R, int a, int b, REAL gm1, REAL out[4])
{
    const REAL wl = (REAL)sqrt((double)L.v[0]), wr = (REAL)sqrt((double)R.v[0]);
    const REAL ual = L.v[a] / L.v[0], ubl = L.v[b] / L.v[0];
    const REAL uar = R.v[a] / R.v[0], ubr = R.v[b] / R.v[0];
    const REAL pl = pressure(L, gm1), pr = pressure(R, gm1);
    const REAL hl = (L.v[3] + pl) / L.v[0], hr = (R.v[3] + pr) / R.v[0];
    const REAL ua = (wl * ual + wr * uar) / (wl + wr);
    const REAL ub = (wl * ubl + wr * ubr) / (wl + wr);
    const REAL H = (wl * hl + wr * hr) / (wl + wr);
    const REAL c2 = gm1 * (H - (REAL)0.5 * (ua * ua + ub * ub));
    out[0] = ua;
    out[1] = ub;
    out[2] = H;
    out[3] = (REAL)fabs((double)ua) + (REAL)sqrt((double)c2);
}

/* Numerical flux through the face between cells B and C of the 1D run
 * A, B, C, D (App. B: pressure-ratio reconstruction, then the Rusanov-form
 * flux).  a selects the normal momentum component; scheme the variant bits.
 * Each cell's pressure ratio is the plain quotient of its forward and
 * backward pressure jumps, and the minmod factor takes the plain reciprocal
 * of that ratio. */
static void face_flux_states(state4 A, state4 B, state4 C, state4 D, int a, REAL gamma, int scheme, REAL out[4],
                             state4* Lo, state4* Ro)
{
    const REAL gm1 = gamma - (REAL)1;
    const int b = (a == 1) ? 2 : 1;
    const int literal = (scheme & SCHEME_LIMITER_LITERAL) != 0;
    const REAL pA = pressure(A, gm1), pB = pressure(B, gm1), pC = pressure(C, gm1), pD = pressure(D, gm1);
    const REAL rB = (pC - pB) / (pB - pA); /* ratio at the left cell  */
    const REAL rC = (pD - pC) / (pC - pB); /* ratio at the right cell */
    state4 L = B, R = C;
    if (ratio_ok(rB)) {
        /* minmod reading: min(1/r_B, 1); as printed: min(r_B, 1) */
        const REAL e = literal ? rB : (REAL)1 / rB;
        const REAL phi = (REAL)0.5 * (e < (REAL)1 ? e : (REAL)1);
        for (int c = 0; c < 4; ++c) L.v[c] = B.v[c] + phi * (C.v[c] - B.v[c]);
    }
    if (ratio_ok(rC)) {
        /* minmod reading: min(r_C, 1); as printed: min(1/r_C, 1) */
        const REAL e = literal ? (REAL)1 / rC : rC;
        const REAL phi = (REAL)0.5 * (e < (REAL)1 ? e : (REAL)1);
        for (int c = 0; c < 4; ++c) R.v[c] = C.v[c] + phi * (B.v[c] - C.v[c]);
    }
    REAL fL[4], fR[4], sL, sR;
    phys_flux(L, a, b, gamma, gm1, fL, &sL);
    phys_flux(R, a, b, gamma, gm1, fR, &sR);
    REAL s = sL > sR ? sL : sR;
    if (scheme & SCHEME_SPEED_ROE) {
        REAL roe[4];
        roe_average(L, R, a, b, gm1, roe);
        s = roe[3];
    }
    for (int c = 0; c < 4; ++c) out[c] = (REAL)0.5 * ((fR[c] + fL[c]) + s * (L.v[c] - R.v[c]));
    if (Lo) *Lo = L;
    if (Ro) *Ro = R;
}

static void face_flux(state4 A, state4 B, state4 C, state4 D, int a, REAL gamma, int scheme, REAL out[4])
{
    face_flux_states(A, B, C, D, a, gamma, scheme, out, 0, 0);
}

/* The reconstructed face states and the numerical flux through the face
 * between cells B and C of the run A, B, C, D (each a 4-vector of conserved
 * variables); a = 1 for an x face, 2 for a y face; scheme the variant bits.
 * Exposed for unit checks of the limiter and flux against their textbook
 * forms. */
void NAME(oracle_face)(const REAL* A, const REAL* B, const REAL* C, const REAL* D, int64_t a, double gamma,
                       int64_t scheme, REAL* Lout, REAL* Rout, REAL* Fout)
{
    state4 s[4];
    const REAL* in[4] = {A, B, C, D};
    for (int k = 0; k < 4; ++k)
        for (int c = 0; c < 4; ++c) s[k].v[c] = in[k][c];
    state4 L, R;
    face_flux_states(s[0], s[1], s[2], s[3], (int)a, (REAL)gamma, (int)scheme, Fout, &L, &R);
    for (int c = 0; c < 4; ++c) { Lout[c] = L.v[c]; Rout[c] = R.v[c]; }
}

/* Roe average of two states (see roe_average), exposed for unit checks. */
void NAME(oracle_roe_average)(const REAL* L, const REAL* R, int64_t a, double gamma, REAL* out)
{
    state4 l, r;
    for (int c = 0; c < 4; ++c) { l.v[c] = L[c]; r.v[c] = R[c]; }
    roe_average(l, r, (int)a, a == 1 ? 2 : 1, (REAL)gamma - (REAL)1, out);
}

/* One RK stage: Qout = Qbase - hx (Fx_{i+1/2} - Fx_{i-1/2}) - hy (Gy_{j+1/2} - Gy_{j-1/2}),
 * fluxes evaluated on Qflux.  Face fluxes are computed once per face into
 * fx / gy (each 4*N*N), so the two cells sharing a face use the same value. */
static void euler_stage(const REAL* Qbase, const REAL* Qflux, REAL* Qout, int64_t N, REAL hx, REAL hy,
                        REAL gamma, int scheme, REAL* fx, REAL* gy)
{
    const int64_t NN = N * N;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < N; ++j) {
        for (int64_t i = 0; i < N; ++i) {
            REAL f[4];
            /* x face i+1/2 of row j: cells i-1, i, i+1, i+2 */
            face_flux(load4(Qflux, NN, j * N + wrap(i - 1, N)), load4(Qflux, NN, j * N + i),
                      load4(Qflux, NN, j * N + wrap(i + 1, N)), load4(Qflux, NN, j * N + wrap(i + 2, N)), 1,
                      gamma, scheme, f);
            for (int c = 0; c < 4; ++c) fx[c * NN + j * N + i] = f[c];
            /* y face j+1/2 of column i: rows j-1, j, j+1, j+2 */
            face_flux(load4(Qflux, NN, wrap(j - 1, N) * N + i), load4(Qflux, NN, j * N + i),
                      load4(Qflux, NN, wrap(j + 1, N) * N + i), load4(Qflux, NN, wrap(j + 2, N) * N + i), 2,
                      gamma, scheme, f);
            for (int c = 0; c < 4; ++c) gy[c * NN + j * N + i] = f[c];
        }
    }
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < N; ++j) {
        for (int64_t i = 0; i < N; ++i) {
            const int64_t k = j * N + i;
            for (int c = 0; c < 4; ++c) {
                const REAL dF = fx[c * NN + k] - fx[c * NN + j * N + wrap(i - 1, N)];
                const REAL dG = gy[c * NN + k] - gy[c * NN + wrap(j - 1, N) * N + i];
                Qout[c * NN + k] = (Qbase[c * NN + k] - hx * dF) - hy * dG;
            }
        }
    }
}

/* Euler walls.  With walls a row has N + 1 faces, f = 0 .. N (face f lies
 * between cells f - 1 and f; faces 0 and N are the two walls), and each face
 * reads the cells f - 2 .. f + 1, where cells outside [0, N) are ghosts:
 *   BC_NEUMANN (zero gradient, transmissive): a ghost holds the edge cell;
 *   BC_REFLECT (slip wall): ghost -1 - k holds cell k (ghost N + k holds
 *     cell N - 1 - k) with the momentum normal to the wall negated.
 * k is the cell index along the face normal, a the normal momentum (1: x,
 * 2: y); (i, j) the cell's other coordinates are given by the caller. */
static inline state4 euler_ghost(const REAL* Q, int64_t NN, int64_t N, int64_t k, int64_t other, int a, int bc)
{
    int64_t kk = k;
    int flip = 0;
    if (k < 0 || k >= N) {
        if (bc == BC_NEUMANN) {
            kk = k < 0 ? 0 : N - 1;
        } else {
            kk = k < 0 ? -1 - k : 2 * N - 1 - k;
            flip = 1;
        }
    }
    state4 s = load4(Q, NN, a == 1 ? other * N + kk : kk * N + other);
    if (flip) s.v[a] = -s.v[a];
    return s;
}

/* One RK stage with walls: faces 0 .. N per row (x) and per column (y),
 * Qout = Qbase - hx (F_{i+1} - F_i) - hy (G_{j+1} - G_j) with face i left
 * of cell i.  fx and gy hold 4*N*(N+1) values each. */
static void euler_stage_walls(const REAL* Qbase, const REAL* Qflux, REAL* Qout, int64_t N, REAL hx, REAL hy,
                              REAL gamma, int scheme, int bc, REAL* fx, REAL* gy)
{
    const int64_t NN = N * N, NF = N * (N + 1);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < N; ++j) {
        for (int64_t f = 0; f <= N; ++f) {
            REAL o[4];
            /* x face f of row j: cells f-2 .. f+1 */
            face_flux(euler_ghost(Qflux, NN, N, f - 2, j, 1, bc), euler_ghost(Qflux, NN, N, f - 1, j, 1, bc),
                      euler_ghost(Qflux, NN, N, f, j, 1, bc), euler_ghost(Qflux, NN, N, f + 1, j, 1, bc), 1, gamma,
                      scheme, o);
            for (int c = 0; c < 4; ++c) fx[c * NF + j * (N + 1) + f] = o[c];
            /* y face f of column j */
            face_flux(euler_ghost(Qflux, NN, N, f - 2, j, 2, bc), euler_ghost(Qflux, NN, N, f - 1, j, 2, bc),
                      euler_ghost(Qflux, NN, N, f, j, 2, bc), euler_ghost(Qflux, NN, N, f + 1, j, 2, bc), 2, gamma,
                      scheme, o);
            for (int c = 0; c < 4; ++c) gy[c * NF + j * (N + 1) + f] = o[c];
        }
    }
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < N; ++j) {
        for (int64_t i = 0; i < N; ++i) {
            const int64_t k = j * N + i;
            for (int c = 0; c < 4; ++c) {
                const REAL dF = fx[c * NF + j * (N + 1) + i + 1] - fx[c * NF + j * (N + 1) + i];
                const REAL dG = gy[c * NF + i * (N + 1) + j + 1] - gy[c * NF + i * (N + 1) + j];
                Qout[c * NN + k] = (Qbase[c * NN + k] - hx * dF) - hy * dG;
            }
        }
    }
}

/* M explicit-midpoint RK2 steps of the 2D Euler equations on an N x N
 * periodic grid with spacings dx, dy.  Q (4*N*N) holds Q^0 on entry and
 * Q^M on exit; work must hold 16*N*N values (Q*, Q^{n+1}, face fluxes);
 * scheme = variant bits (0: minmod + Rusanov). */
void NAME(oracle_euler_run_bc)(REAL* Q, REAL* work, int64_t N, double dt, double dx, double dy, double gamma_in,
                               int64_t M, int64_t scheme, int64_t bc)
{
    const int64_t NN = N * N, NF = N * (N + 1);
    REAL* qs = work;
    REAL* qn = work + 4 * NN;
    REAL* fx = work + 8 * NN;
    REAL* gy = fx + 4 * NF;
    const REAL gamma = (REAL)gamma_in;
    const REAL hx = (REAL)(0.5 * dt / dx), hy = (REAL)(0.5 * dt / dy);
    const REAL kx = (REAL)(dt / dx), ky = (REAL)(dt / dy);
    for (int64_t m = 0; m < M; ++m) {
        if (bc == BC_PERIODIC) {
            euler_stage(Q, Q, qs, N, hx, hy, gamma, (int)scheme, fx, gy);
            euler_stage(Q, qs, qn, N, kx, ky, gamma, (int)scheme, fx, gy);
        } else {
            euler_stage_walls(Q, Q, qs, N, hx, hy, gamma, (int)scheme, (int)bc, fx, gy);
            euler_stage_walls(Q, qs, qn, N, kx, ky, gamma, (int)scheme, (int)bc, fx, gy);
        }
        memcpy(Q, qn, (size_t)(4 * NN) * sizeof(REAL));
    }
}

/* Periodic run. */
void NAME(oracle_euler_run)(REAL* Q, REAL* work, int64_t N, double dt, double dx, double dy, double gamma_in,
                            int64_t M, int64_t scheme)
{
    NAME(oracle_euler_run_bc)(Q, work, N, dt, dx, dy, gamma_in, M, scheme, BC_PERIODIC);
}

/* Work size, in values, that oracle_euler_run(_bc) needs. */
int64_t NAME(oracle_euler_work_values)(int64_t N) { return 16 * N * N + 8 * N; }

/* Stable time step for a CFL number: dt = cfl / max_cells((|u|+c)/dx + (|v|+c)/dy),
 * evaluated in double from the (exactly widened) state.  Not in the paper,
 * which states no time step. */
double NAME(oracle_cfl_dt)(const REAL* Q, int64_t N, double dx, double dy, double gamma, double cfl)
{
    const int64_t NN = N * N;
    double smax = 0.0;
    for (int64_t k = 0; k < NN; ++k) {
        const double rho = (double)Q[k], m = (double)Q[NN + k], n = (double)Q[2 * NN + k],
                     E = (double)Q[3 * NN + k];
        const double u = m / rho, v = n / rho;
        const double p = (gamma - 1.0) * (E - 0.5 * (m * u + n * v));
        const double c = sqrt(gamma * p / rho);
        const double s = (fabs(u) + c) / dx + (fabs(v) + c) / dy;
        if (s > smax) smax = s;
    }
    return cfl / smax;
}

/* Per-plane sums in double, sequential order: the conserved totals
 * (sum rho, sum rho u, sum rho v, sum E; or sum T for heat). */
void NAME(oracle_plane_sums)(const REAL* Q, int64_t nvar, int64_t NN, double* out)
{
    for (int64_t c = 0; c < nvar; ++c) {
        double s = 0.0;
        for (int64_t k = 0; k < NN; ++k) s += (double)Q[c * NN + k];
        out[c] = s;
    }
}
