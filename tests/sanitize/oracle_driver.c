/* Runs every entry point of the oracle on small grids, for the address and
 * undefined-behaviour sanitizer build of tests/test_sanitizers.py.  The
 * values are not checked here (the pinned tests do that); the run must end
 * without a sanitizer report. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#define DECL(T, S)                                                                                              \
    void oracle_heat_run_bc##S(T* T_, T* work, int64_t N, double r, int64_t M, int64_t bc, double bcv);        \
    void oracle_heat_adjoint_bc##S(const T* T0, const T* g, T* gT0, double* dJdr, int64_t N, double r,         \
                                   int64_t M, T* levels, T* work, int64_t bc, double bcv);                     \
    void oracle_heat_adjoint##S(const T* T0, const T* g, T* gT0, double* dJdr, int64_t N, double r, int64_t M,  \
                                T* levels, T* work);                                                            \
    double oracle_l2_mismatch##S(const T* T_, const T* Ts, int64_t n);                                         \
    void oracle_euler_run_bc##S(T* Q, T* work, int64_t N, double dt, double dx, double dy, double gamma,        \
                                int64_t M, int64_t scheme, int64_t bc);                                        \
    int64_t oracle_euler_work_values##S(int64_t N);                                                            \
    double oracle_cfl_dt##S(const T* Q, int64_t N, double dx, double dy, double gamma, double cfl);            \
    void oracle_plane_sums##S(const T* Q, int64_t nvar, int64_t NN, double* out);

DECL(double, _f64)
DECL(float, _f32)

#define RUN(T, S)                                                                                      \
    do {                                                                                               \
        const int64_t N = 24, NN = N * N;                                                              \
        T* a = calloc(NN, sizeof(T));                                                                  \
        T* b = calloc(NN, sizeof(T));                                                                  \
        T* g = calloc(NN, sizeof(T));                                                                  \
        T* w = calloc(NN, sizeof(T));                                                                  \
        T* lv = calloc(8 * NN, sizeof(T));                                                             \
        for (int64_t k = 0; k < NN; ++k) {                                                             \
            a[k] = (T)sin(0.37 * k);                                                                   \
            g[k] = (T)cos(0.11 * k);                                                                   \
        }                                                                                              \
        double d = 0.0, s4[4];                                                                         \
        for (int64_t bc = 0; bc < 3; ++bc) {                                                           \
            for (int64_t k = 0; k < NN; ++k) b[k] = a[k];                                              \
            oracle_heat_run_bc##S(b, w, N, 0.2, 7, bc, 0.5);                                           \
            oracle_heat_adjoint_bc##S(a, g, b, &d, N, 0.2, 5, lv, w, bc, 0.5);                         \
        }                                                                                              \
        oracle_heat_adjoint##S(a, g, b, &d, N, 0.2, 6, lv, w);                                         \
        d += oracle_l2_mismatch##S(a, g, NN);                                                          \
        T* q = calloc(4 * NN, sizeof(T));                                                              \
        T* qw = calloc(oracle_euler_work_values##S(N), sizeof(T));                                     \
        for (int64_t scheme = 0; scheme < 4; ++scheme)                                                 \
            for (int64_t bc = 0; bc < 4; bc += (bc == 0 ? 2 : 1)) {                                    \
                for (int64_t k = 0; k < NN; ++k) {                                                     \
                    q[k] = (T)(1.0 + 0.1 * sin(0.3 * k));                                              \
                    q[NN + k] = (T)(0.2 * cos(0.2 * k));                                               \
                    q[2 * NN + k] = (T)(0.1 * sin(0.5 * k));                                           \
                    q[3 * NN + k] = (T)(2.5 + 0.05 * cos(0.7 * k));                                    \
                }                                                                                      \
                d += oracle_cfl_dt##S(q, N, 0.4, 0.4, 1.4, 0.4);                                       \
                oracle_euler_run_bc##S(q, qw, N, 0.01, 0.4, 0.4, 1.4, 3, scheme, bc);                  \
                oracle_plane_sums##S(q, 4, NN, s4);                                                    \
                d += s4[0];                                                                            \
            }                                                                                          \
        printf(#S " %g\n", d);                                                                         \
        free(a), free(b), free(g), free(w), free(lv), free(q), free(qw);                               \
    } while (0)

int main(void)
{
    RUN(double, _f64);
    RUN(float, _f32);
    return 0;
}
