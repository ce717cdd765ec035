// capi.cpp -- the C ABI of libswept (declared in include/swept.h): argument
// validation, the phase plan of the swept rule, workspace layout and the
// launch sequences.  Validation never touches the HIP runtime, so every
// error path is testable without a GPU.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

#include "../../include/swept.h"
#include "hetero.h"
#include "launch.h"

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

int hip_fail(hipError_t e, const char* what)
{
    (void)hipGetLastError();  // reported here: do not let it resurface at the caller's next HIP call
    return fail(SWEPT_EHIP, "%s: %s", what, hipGetErrorString(e));
}

constexpr size_t kAlign = 256;
constexpr int kParts = 1024;          // reduction partials per plane
constexpr size_t kLdsMax = 160 * 1024; // gfx950 LDS per workgroup

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Derived {
    int nvar, n, lps, tile, h, wg;
    size_t scalar, state_bytes, lds_bytes;
    double r, dx, dy;
};

// LDS of one swept workgroup: heat keeps two level-parity windows; Euler
// also a pressure plane (kernels.hip, euler_level).
size_t phase_lds(int nvar, int n, int tile, size_t scalar)
{
    if (nvar == 1) {
        const size_t W = (size_t)tile + 2 * n;
        return 2 * W * (W + swept::kHeatPad) * scalar;
    }
    return swept::euler_phase_lds(scalar == 8 ? 0 : 1, tile);
}

bool tile_ok(int N, int tile, int n, int nvar, size_t scalar)
{
    return tile > 2 * n && tile % (2 * n) == 0 && N % tile == 0 && N >= 2 * tile &&
           phase_lds(nvar, n, tile, scalar) <= kLdsMax;
}

int default_tile(const swept_problem* p, int n, int nvar, size_t scalar)
{
    static const int heat_order[] = {64, 32, 16, 8, 0};
    static const int e64_order[] = {16, 32, 8, 0};
    static const int e32_order[] = {16, 32, 8, 0};
    const int* order = p->kind == SWEPT_HEAT ? heat_order : (p->dtype == SWEPT_F64 ? e64_order : e32_order);
    for (int k = 0; order[k]; ++k)
        if (tile_ok(p->nx, order[k], n, nvar, scalar)) return order[k];
    return 0;
}

int derive(const swept_problem* p, const swept_tuning* t, Derived* d)
{
    if (!p) return fail(SWEPT_EINVAL, "problem is NULL");
    if (p->kind != SWEPT_HEAT && p->kind != SWEPT_EULER) return fail(SWEPT_EINVAL, "unknown kind %d", p->kind);
    if (p->dtype != SWEPT_F64 && p->dtype != SWEPT_F32) return fail(SWEPT_EINVAL, "unknown dtype %d", p->dtype);
    if (p->nx <= 0 || p->ny <= 0) return fail(SWEPT_ESHAPE, "grid %d x %d is empty", p->nx, p->ny);
    if (p->nx != p->ny) return fail(SWEPT_ESHAPE, "grid must be square (nx=%d, ny=%d)", p->nx, p->ny);
    if (p->nx > 32768) return fail(SWEPT_ESHAPE, "nx=%d exceeds 32768", p->nx);
    if (!(p->lx > 0) || !(p->ly > 0) || !std::isfinite(p->lx) || !std::isfinite(p->ly))
        return fail(SWEPT_EINVAL, "domain lengths must be positive");
    if (!(p->dt > 0) || !std::isfinite(p->dt)) return fail(SWEPT_EUNSTABLE, "dt must be positive (dt=%g)", p->dt);
    if (p->boundary < SWEPT_BC_PERIODIC || p->boundary > SWEPT_BC_REFLECT)
        return fail(SWEPT_EINVAL, "unknown boundary %d", p->boundary);
    if (p->kind == SWEPT_HEAT && p->boundary == SWEPT_BC_REFLECT)
        return fail(SWEPT_EINVAL, "heat has no slip wall (use SWEPT_BC_NEUMANN)");
    if (p->kind == SWEPT_EULER && p->boundary == SWEPT_BC_DIRICHLET)
        return fail(SWEPT_ENOTSUP, "Euler walls are SWEPT_BC_NEUMANN (zero gradient) or SWEPT_BC_REFLECT");
    if (!std::isfinite(p->boundary_value)) return fail(SWEPT_EINVAL, "boundary value must be finite");
    if (p->scheme & ~(SWEPT_LIMITER_LITERAL | SWEPT_SPEED_ROE))
        return fail(SWEPT_EINVAL, "unknown scheme bits %d", p->scheme);
    if (p->kind == SWEPT_HEAT && p->scheme != 0) return fail(SWEPT_EINVAL, "heat has no scheme variants");
    d->nvar = p->kind == SWEPT_HEAT ? 1 : 4;
    d->n = p->kind == SWEPT_HEAT ? 1 : 2;
    d->lps = p->kind == SWEPT_HEAT ? 1 : 2;
    d->scalar = p->dtype == SWEPT_F64 ? 8 : 4;
    d->dx = p->lx / p->nx;
    d->dy = p->ly / p->ny;
    d->r = 0.0;
    if (p->kind == SWEPT_HEAT) {
        if (!(p->alpha > 0) || !std::isfinite(p->alpha)) return fail(SWEPT_EINVAL, "alpha must be positive");
        if (d->dx != d->dy) return fail(SWEPT_ESHAPE, "heat needs dx == dy");
        d->r = p->alpha * p->dt / (d->dx * d->dx);
        if (4.0 * d->r > 1.0) return fail(SWEPT_EUNSTABLE, "heat: 4r = %g > 1 is unstable", 4.0 * d->r);
    } else {
        if (!(p->gamma > 1) || !std::isfinite(p->gamma)) return fail(SWEPT_EINVAL, "gamma must exceed 1");
    }
    int tile = t ? t->tile : 0;
    if (tile == 0) {
        tile = default_tile(p, d->n, d->nvar, d->scalar);
        if (tile == 0) return fail(SWEPT_ESHAPE, "no supported tile for nx=%d", p->nx);
    }
    if (tile <= 2 * d->n || tile % (2 * d->n) != 0)
        return fail(SWEPT_ESHAPE, "tile %d must be a multiple of 2n=%d and larger than it", tile, 2 * d->n);
    if (p->nx % tile != 0) return fail(SWEPT_ESHAPE, "nx=%d is not divisible by tile %d", p->nx, tile);
    if (p->nx < 2 * tile) return fail(SWEPT_ESHAPE, "nx=%d must be at least 2*tile=%d", p->nx, 2 * tile);
    d->lds_bytes = phase_lds(d->nvar, d->n, tile, d->scalar);
    if (d->lds_bytes > kLdsMax)
        return fail(SWEPT_ESHAPE, "tile %d needs %zu bytes of LDS (max %zu)", tile, d->lds_bytes, kLdsMax);
    int wg = t ? t->wg : 0;
    if (wg == 0) wg = 256;
    const int wg_max = 1024;
    if (wg < 64 || wg > wg_max || wg % 64 != 0)
        return fail(SWEPT_EINVAL, "wg=%d must be a multiple of 64 in [64,%d]", wg, wg_max);
    d->tile = tile;
    d->h = tile / (2 * d->n);
    d->wg = wg;
    d->state_bytes = (size_t)d->nvar * p->nx * p->ny * d->scalar;
    return SWEPT_OK;
}

size_t table_bytes(const Derived& d) { return sizeof(swept::LevelEntry) * swept::level_table_entries(d.h); }

size_t workspace_for(const Derived& d)
{
    return align_up(d.state_bytes) + align_up(sizeof(double) * 4 * kParts) + align_up(sizeof(double) * 4) +
           align_up(table_bytes(d));
}

// ---- adjoint tape (heat): checkpoints, scratch pairs, remainder stash, partial sums
struct TapePlan {
    int64_t cycles, rem;  // n_steps = cycles*h + rem
    int64_t nck;          // checkpoints: one per cycle start, plus the remainder's start
    int pk_max;           // packed forward levels per reverse workgroup
    int std_blocks;       // blocks of the remainder's one-step adjoint kernel
    size_t ck_off, strips_off, pairs_off, stash_off, part_off, total;
    int64_t nparts;
};

constexpr int kStdAdjBlocks = 1024;
constexpr int kAdjCombine = 512;  // first-stage blocks of the pairing sum (fixed chunks, fixed order)

int tape_plan(const Derived& d, int nx, int64_t n_steps, TapePlan* t)
{
    const int h = d.h, tiles = nx / d.tile;
    t->cycles = n_steps / h;
    t->rem = n_steps % h;
    t->nck = t->cycles + (t->rem > 0 ? 1 : 0);
    t->pk_max = 4 * (h - 1) * h * (2 * h - 1) / 6;  // sum_{j<h} (2j)^2: the largest recomputed footprint
    t->std_blocks = kStdAdjBlocks;
    const size_t S = align_up(d.state_bytes), SL = align_up(sizeof(double) * (size_t)nx * nx);
    t->ck_off = 0;
    // per cycle, the forward's Up-Pyramid strips (P0 P1) and Bridge strips (Q0 Q1), kept so that
    // the reverse sweep need not recompute them
    t->strips_off = t->ck_off + S * (size_t)t->nck;
    t->pairs_off = t->strips_off + 4 * S * (size_t)t->cycles;
    t->stash_off = t->pairs_off + 2 * SL;  // L0 L1 (lambda, double)
    t->part_off = t->stash_off + S * (size_t)t->rem;
    t->nparts = t->cycles * 4 * (int64_t)tiles * tiles + t->rem * kStdAdjBlocks;
    t->total = t->part_off + align_up(sizeof(double) * (size_t)(t->nparts + 1 + kAdjCombine));
    return SWEPT_OK;
}

int half_width_host(int t, int h, int n)
{
    if (t < 1 || t > 2 * h - 1) return 0;
    return n * (t < 2 * h - t ? t : 2 * h - t);
}

// Host copy of the per-level table (see launch.h).  t is the level within
// the shape's window; Bridges' shrinking axis is at t + h.
// Fewest rows per heat strip: a strip's set-up is paid once for all its rows.
constexpr int kMinRows = 1;

void build_level_table(const Derived& d, swept::LevelEntry* tab)
{
    const int h = d.h, n = d.n, C = d.tile / 2 + n;
    for (int k = 0; k < swept::level_table_entries(h); ++k) tab[k] = swept::LevelEntry{};
    auto fill = [&](swept::LevelEntry& e, int hx, int hy, int hx2, int hy2) {
        e.x0 = C - hx;
        e.y0 = C - hy;
        e.fw = 2 * hx;
        e.fh = 2 * hy;
        e.pw = hx;  // fw is even: pairs of columns
        const int pairs = e.pw * e.fh;
        e.R = std::max((pairs + d.wg - 1) / d.wg, std::min(kMinRows, e.fh));
        e.spc = (e.fh + e.R - 1) / e.R;
        e.hx2 = hx2;
        e.hy2 = hy2;
        e.inv_fw = e.fw > 0 ? 1.0f / (float)e.fw : 0.0f;
        e.inv_pw = e.pw > 0 ? 1.0f / (float)e.pw : 0.0f;
    };
    for (int t = 1; t <= 2 * h - 1; ++t) {  // Octahedron
        const int hw = half_width_host(t, h, n), hw2 = half_width_host(t + 2, h, n);
        fill(tab[t], hw, hw, hw2, hw2);
    }
    for (int t = 1; t <= h - 1; ++t) {  // Bridges: growing axis t, shrinking axis t + h
        const int g = half_width_host(t, h, n), s = half_width_host(t + h, h, n);
        const bool has2 = t + 2 <= h - 1;
        const int g2 = has2 ? half_width_host(t + 2, h, n) : 0, s2 = has2 ? half_width_host(t + 2 + h, h, n) : 0;
        fill(tab[2 * h + t], g, s, g2, s2);  // X-Bridge (w, w-1): x grows
        fill(tab[3 * h + t], s, g, s2, g2);  // Y-Bridge (w-1, w): y grows
    }
}

}  // namespace

struct swept_ctx {
    swept_problem prob;
    Derived d;
    void* state;
    void* work;
    size_t work_bytes;
    hipStream_t stream;
    void* buf1;
    double* partials;
    double* red;
    double c[5];  // scheme constants (see PhaseArgs)
    int std_ts;
    swept::LevelEntry* tab_dev;  // level table inside the workspace
    size_t adj_lds;              // LDS of an adjoint workgroup (0: adjoint unavailable)
};

extern "C" {

const char* swept_last_error(void) { return g_err; }

int swept_workspace_bytes(const swept_problem* prob, const swept_tuning* tune, size_t* bytes)
{
    if (!bytes) return fail(SWEPT_EINVAL, "bytes is NULL");
    Derived d;
    const int rc = derive(prob, tune, &d);
    if (rc) return rc;
    *bytes = workspace_for(d);
    return SWEPT_OK;
}

int swept_init(swept_ctx** ctx, const swept_problem* prob, const swept_tuning* tune, void* d_state, void* d_work,
               size_t work_bytes, void* hip_stream)
{
    if (!ctx) return fail(SWEPT_EINVAL, "ctx is NULL");
    *ctx = nullptr;
    Derived d;
    int rc = derive(prob, tune, &d);
    if (rc) return rc;
    if (!d_state) return fail(SWEPT_EINVAL, "state pointer is NULL");
    if (!d_work) return fail(SWEPT_EINVAL, "workspace pointer is NULL");
    if ((reinterpret_cast<uintptr_t>(d_state) | reinterpret_cast<uintptr_t>(d_work)) % 16 != 0)
        return fail(SWEPT_EINVAL, "state and workspace must be 16-byte aligned");
    const size_t need = workspace_for(d);
    if (work_bytes < need) return fail(SWEPT_EWORKSPACE, "workspace %zu bytes < %zu needed", work_bytes, need);
    swept_ctx* c = new (std::nothrow) swept_ctx();
    if (!c) return fail(SWEPT_EINVAL, "out of host memory");
    c->prob = *prob;
    c->d = d;
    c->state = d_state;
    c->work = d_work;
    c->work_bytes = work_bytes;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    char* w = static_cast<char*>(d_work);
    c->buf1 = w;
    c->partials = reinterpret_cast<double*>(w + align_up(d.state_bytes));
    c->red = reinterpret_cast<double*>(w + align_up(d.state_bytes) + align_up(sizeof(double) * 4 * kParts));
    if (prob->kind == SWEPT_HEAT) {
        c->c[0] = d.r;
        c->c[1] = prob->boundary == SWEPT_BC_DIRICHLET ? prob->boundary_value : 0.0;
        c->c[2] = c->c[3] = c->c[4] = 0.0;
    } else {
        c->c[0] = prob->gamma;
        c->c[1] = 0.5 * prob->dt / d.dx;
        c->c[2] = 0.5 * prob->dt / d.dy;
        c->c[3] = prob->dt / d.dx;
        c->c[4] = prob->dt / d.dy;
    }
    // fused Euler step tile: the largest of 16, 8, 4 dividing nx (nx is a multiple of 4 for Euler)
    // whose window (tile + 4-cell halo) is at most nx wide, so a window meets the domain edge at
    // most once (the walls substitute ghost cells at that one edge)
    c->std_ts = (prob->nx % 16 == 0 && prob->nx >= 24) ? 16 : (prob->nx % 8 == 0 && prob->nx >= 16) ? 8 : 4;
    c->tab_dev = reinterpret_cast<swept::LevelEntry*>(w + align_up(d.state_bytes) +
                                                      align_up(sizeof(double) * 4 * kParts) +
                                                      align_up(sizeof(double) * 4));
    // the dynamic-LDS ceiling is per kernel, shared by all contexts: always raise it to the maximum
    hipError_t e = swept::set_phase_lds_limit(prob->kind, prob->dtype, kLdsMax);
    if (e == hipSuccess && prob->kind == SWEPT_EULER) e = swept::set_euler_standard_lds_limit(prob->dtype, kLdsMax);
    if (e != hipSuccess) {
        delete c;
        return hip_fail(e, "hipFuncSetAttribute");
    }
    c->adj_lds = 0;
    if (prob->kind == SWEPT_HEAT) {
        const int h = d.h, pk_max = 4 * (h - 1) * h * (2 * h - 1) / 6;
        const size_t lds = swept::adjoint_lds(prob->dtype, d.tile, pk_max, d.wg);
        if (lds <= kLdsMax) {
            c->adj_lds = lds;
            e = swept::set_adjoint_lds_limit(prob->dtype, kLdsMax);
            if (e != hipSuccess) {
                delete c;
                return hip_fail(e, "hipFuncSetAttribute");
            }
        }
    }
    {
        const int ne = swept::level_table_entries(d.h);
        swept::LevelEntry* host = new (std::nothrow) swept::LevelEntry[ne];
        if (!host) {
            delete c;
            return fail(SWEPT_EINVAL, "out of host memory");
        }
        build_level_table(d, host);
        e = hipMemcpyAsync(c->tab_dev, host, table_bytes(d), hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        delete[] host;
        if (e != hipSuccess) {
            delete c;
            return hip_fail(e, "level table upload");
        }
    }
    *ctx = c;
    return SWEPT_OK;
}

int swept_query(const swept_ctx* c, swept_info* info)
{
    if (!c || !info) return fail(SWEPT_EINVAL, "NULL argument");
    info->nvar = c->d.nvar;
    info->n = c->d.n;
    info->levels_per_step = c->d.lps;
    info->tile = c->d.tile;
    info->h = c->d.h;
    info->wg = c->d.wg;
    info->r = c->d.r;
    info->dx = c->d.dx;
    info->dy = c->d.dy;
    info->state_bytes = c->d.state_bytes;
    info->lds_bytes = c->d.lds_bytes;
    return SWEPT_OK;
}

int swept_set_stream(swept_ctx* c, void* hip_stream)
{
    if (!c) return fail(SWEPT_EINVAL, "ctx is NULL");
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    return SWEPT_OK;
}

static swept::PhaseArgs phase_args(const swept_ctx* c, int L)
{
    swept::PhaseArgs a{};
    a.buf0 = a.out0 = c->state;
    a.buf1 = a.out1 = c->buf1;
    a.lvl0 = c->state;
    a.N = c->prob.nx;
    a.tile = c->d.tile;
    a.h = c->d.h;
    a.tiles = c->prob.nx / c->d.tile;
    a.L = L;
    a.tab = c->tab_dev;
    a.scheme = c->prob.scheme;
    a.bc = c->prob.boundary;
    for (int k = 0; k < 5; ++k) a.p[k] = c->c[k];
    return a;
}

// Swept advance of n_steps on the context's state, flat to flat.
static int advance_impl(swept_ctx* c, int64_t n_steps)
{
    if (n_steps == 0) return SWEPT_OK;
    const int64_t L64 = n_steps * c->d.lps;
    if (L64 > (int64_t)1 << 30) return fail(SWEPT_EINVAL, "n_steps too large");
    const int L = (int)L64;
    const int W = (L + c->d.h - 1) / c->d.h;
    swept::PhaseArgs a = phase_args(c, L);
    for (int ph = 0; ph <= 2 * W; ++ph) {
        a.phase = ph;
        hipError_t e = swept::launch_phase(c->prob.kind, c->prob.dtype, a, c->d.wg, c->d.lds_bytes, c->stream);
        if (e != hipSuccess) return hip_fail(e, "swept phase launch");
    }
    if (L & 1) {  // level L lives in buffer 1
        hipError_t e = hipMemcpyAsync(c->state, c->buf1, c->d.state_bytes, hipMemcpyDeviceToDevice, c->stream);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
    }
    return SWEPT_OK;
}

int swept_advance(swept_ctx* c, int64_t n_steps)
{
    if (!c) return fail(SWEPT_EINVAL, "ctx is NULL");
    if (n_steps < 0) return fail(SWEPT_EINVAL, "n_steps=%lld < 0", (long long)n_steps);
    return advance_impl(c, n_steps);
}

static int tape_check(const swept_ctx* c, int64_t n_steps, TapePlan* t)
{
    if (!c) return fail(SWEPT_EINVAL, "ctx is NULL");
    if (c->prob.kind != SWEPT_HEAT) return fail(SWEPT_ENOTSUP, "the adjoint is implemented for heat only");
    if (n_steps < 0) return fail(SWEPT_EINVAL, "n_steps=%lld < 0", (long long)n_steps);
    if (c->adj_lds == 0)
        return fail(SWEPT_ESHAPE, "tile %d too large for the adjoint's LDS (all levels of a shape are kept)",
                    c->d.tile);
    return tape_plan(c->d, c->prob.nx, n_steps, t);
}

int swept_tape_bytes(const swept_ctx* c, int64_t n_steps, size_t* bytes)
{
    if (!bytes) return fail(SWEPT_EINVAL, "bytes is NULL");
    TapePlan t;
    const int rc = tape_check(c, n_steps, &t);
    if (rc) return rc;
    *bytes = t.total;
    return SWEPT_OK;
}

int swept_advance_checkpointed(swept_ctx* c, int64_t n_steps, void* d_tape, size_t tape_bytes)
{
    TapePlan t;
    int rc = tape_check(c, n_steps, &t);
    if (rc) return rc;
    if (!d_tape) return fail(SWEPT_EINVAL, "tape is NULL");
    if (tape_bytes < t.total) return fail(SWEPT_EWORKSPACE, "tape %zu bytes < %zu needed", tape_bytes, t.total);
    char* tape = static_cast<char*>(d_tape);
    const size_t S = align_up(c->d.state_bytes);
    const int h = c->d.h;
    for (int64_t k = 0; k < t.nck; ++k) {
        hipError_t e = hipMemcpyAsync(tape + t.ck_off + S * k, c->state, c->d.state_bytes, hipMemcpyDeviceToDevice,
                                      c->stream);
        if (e != hipSuccess) return hip_fail(e, "checkpoint copy");
        if (k == t.cycles) {  // the remainder: a plain advance
            rc = advance_impl(c, t.rem);
            if (rc) return rc;
            continue;
        }
        // one flat-to-flat cycle of h steps: Up-Pyramid strips -> P, Bridge strips -> Q (both kept
        // on the tape), then the first Octahedron, clipped at h, from P, Q and the flat state
        char* pq = tape + t.strips_off + 4 * S * (size_t)k;
        swept::PhaseArgs a = phase_args(c, h);
        a.buf0 = a.out0 = pq;
        a.buf1 = a.out1 = pq + S;
        a.phase = 0;
        e = swept::launch_phase(c->prob.kind, c->prob.dtype, a, c->d.wg, c->d.lds_bytes, c->stream);
        if (e != hipSuccess) return hip_fail(e, "taped Up-Pyramid");
        a.out0 = pq + 2 * S;
        a.out1 = pq + 3 * S;
        a.phase = 1;
        e = swept::launch_phase(c->prob.kind, c->prob.dtype, a, c->d.wg, c->d.lds_bytes, c->stream);
        if (e != hipSuccess) return hip_fail(e, "taped Bridges");
        a.q0 = pq + 2 * S;
        a.q1 = pq + 3 * S;
        a.out0 = c->state;
        a.out1 = c->buf1;
        a.phase = 2;
        e = swept::launch_phase(c->prob.kind, c->prob.dtype, a, c->d.wg, c->d.lds_bytes, c->stream);
        if (e != hipSuccess) return hip_fail(e, "taped Octahedron");
        if (h & 1) {  // level h lives in buffer 1
            e = hipMemcpyAsync(c->state, c->buf1, c->d.state_bytes, hipMemcpyDeviceToDevice, c->stream);
            if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
        }
    }
    return SWEPT_OK;
}

int swept_adjoint(swept_ctx* c, int64_t n_steps, void* d_tape, size_t tape_bytes, const void* d_gTM, void* d_gT0,
                  double* dJ_dalpha)
{
    TapePlan t;
    int rc = tape_check(c, n_steps, &t);
    if (rc) return rc;
    if (!d_tape || !d_gTM || !d_gT0 || !dJ_dalpha) return fail(SWEPT_EINVAL, "NULL argument");
    if (tape_bytes < t.total) return fail(SWEPT_EWORKSPACE, "tape %zu bytes < %zu needed", tape_bytes, t.total);
    char* tape = static_cast<char*>(d_tape);
    const size_t S = align_up(c->d.state_bytes), SB = c->d.state_bytes;
    auto ck = [&](int64_t k) { return static_cast<void*>(tape + t.ck_off + S * k); };
    const size_t SL = align_up(sizeof(double) * (size_t)c->prob.nx * c->prob.nx);
    void* La = tape + t.pairs_off;  // lambda (double) at the start of the next reverse step / cycle
    void* Lb = tape + t.pairs_off + SL;
    double* parts = reinterpret_cast<double*>(tape + t.part_off);
    const int N = c->prob.nx, tiles = N / c->d.tile, t2 = tiles * tiles, h = c->d.h;
    hipStream_t st = c->stream;
    const size_t NN = (size_t)N * N;
    hipError_t e = swept::launch_lambda_convert(c->prob.dtype, d_gTM, La, NN, true, st);
    if (e != hipSuccess) return hip_fail(e, "adjoint seed");
    int64_t pslot = 0;
    if (t.rem > 0) {  // the last rem steps: forward levels into the stash, then one adjoint step per level
        char* stash = tape + t.stash_off;
        e = hipMemcpyAsync(stash, ck(t.cycles), SB, hipMemcpyDeviceToDevice, st);
        for (int64_t m = 1; m < t.rem && e == hipSuccess; ++m)
            e = swept::launch_heat_standard(c->prob.dtype, stash + S * (m - 1), stash + S * m, N, c->d.r,
                                            c->prob.boundary, c->c[1], st);
        for (int64_t m = t.rem - 1; m >= 0 && e == hipSuccess; --m) {
            e = swept::launch_adjoint_step(c->prob.dtype, La, Lb, stash + S * m, N, c->d.r, c->prob.boundary,
                                           c->c[1], parts + pslot, t.std_blocks, st);
            pslot += t.std_blocks;
            void* tmp = La;
            La = Lb;
            Lb = tmp;
        }
        if (e != hipSuccess) return hip_fail(e, "adjoint remainder");
    }
    for (int64_t cyc = t.cycles - 1; cyc >= 0; --cyc) {
        // the cycle's forward strips, kept by the checkpointed advance: Up-Pyramid (P), Bridges (Q)
        char* pq = tape + t.strips_off + 4 * S * (size_t)cyc;
        void* P0 = pq;
        void* P1 = pq + S;
        void* Q0 = pq + 2 * S;
        void* Q1 = pq + 3 * S;
        // reverse phases on the other tiling
        swept::PhaseArgs a = phase_args(c, h);
        a.buf0 = P0;
        a.buf1 = P1;
        a.q0 = Q0;
        a.q1 = Q1;
        a.lvl0 = ck(cyc);
        a.lam0 = La;
        a.lam1 = Lb;
        a.shift = 1;
        for (int ph = 0; ph <= 2; ++ph) {
            a.phase = ph;
            a.partials = parts + pslot;
            pslot += (ph & 1) ? 2 * t2 : t2;
            e = swept::launch_adjoint_phase(c->prob.dtype, a, t.pk_max, c->d.wg, c->adj_lds, st);
            if (e != hipSuccess) return hip_fail(e, "adjoint phase launch");
        }
        if (h & 1) {  // lambda of the cycle start lives in the odd buffer
            void* tmp = La;
            La = Lb;
            Lb = tmp;
        }
    }
    e = swept::launch_lambda_convert(c->prob.dtype, La, d_gT0, NN, false, st);
    if (e == hipSuccess)
        e = swept::launch_plane_sums(0, parts, 1, (size_t)pslot, parts + t.nparts + 1, kAdjCombine, parts + t.nparts,
                                     st);
    double dJdr = 0.0;
    if (e == hipSuccess) e = hipMemcpyAsync(&dJdr, parts + t.nparts, sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "adjoint finish");
    *dJ_dalpha = dJdr * c->prob.dt / (c->d.dx * c->d.dx);
    return SWEPT_OK;
}

int standard_advance(swept_ctx* c, int64_t n_steps)
{
    if (!c) return fail(SWEPT_EINVAL, "ctx is NULL");
    if (n_steps < 0) return fail(SWEPT_EINVAL, "n_steps=%lld < 0", (long long)n_steps);
    void* bufs[2] = {c->state, c->buf1};
    for (int64_t m = 0; m < n_steps; ++m) {
        const void* in = bufs[m & 1];
        void* out = bufs[(m + 1) & 1];
        hipError_t e;
        if (c->prob.kind == SWEPT_HEAT) {
            e = swept::launch_heat_standard(c->prob.dtype, in, out, c->prob.nx, c->d.r, c->prob.boundary, c->c[1],
                                            c->stream);
        } else {
            swept::StdArgs a;
            a.N = c->prob.nx;
            a.ts = c->std_ts;
            a.scheme = c->prob.scheme;
            a.bc = c->prob.boundary;
            for (int k = 0; k < 5; ++k) a.p[k] = c->c[k];
            e = swept::launch_euler_standard(c->prob.dtype, in, out, a, c->stream);
        }
        if (e != hipSuccess) return hip_fail(e, "standard step launch");
    }
    if (n_steps & 1) {
        hipError_t e = hipMemcpyAsync(c->state, c->buf1, c->d.state_bytes, hipMemcpyDeviceToDevice, c->stream);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
    }
    return SWEPT_OK;
}

int swept_conserved(swept_ctx* c, double* out)
{
    if (!c || !out) return fail(SWEPT_EINVAL, "NULL argument");
    const size_t NN = (size_t)c->prob.nx * c->prob.ny;
    hipError_t e = swept::launch_plane_sums(c->prob.dtype, c->state, c->d.nvar, NN, c->partials, kParts, c->red,
                                            c->stream);
    if (e != hipSuccess) return hip_fail(e, "plane sums");
    e = hipMemcpyAsync(out, c->red, sizeof(double) * c->d.nvar, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "plane sums copy");
    for (int k = 0; k < c->d.nvar; ++k)
        if (!std::isfinite(out[k])) return fail(SWEPT_ENONFINITE, "sum of plane %d is not finite", k);
    return SWEPT_OK;
}

// Validation shared by both CFL entry points (no HIP call).
static int cfl_check(const swept_problem* prob, const void* d_state, double cfl, double* dt_out, swept_problem* q,
                     Derived* d)
{
    if (!prob || !d_state || !dt_out) return fail(SWEPT_EINVAL, "NULL argument");
    if (prob->kind != SWEPT_EULER) return fail(SWEPT_ENOTSUP, "CFL time step is defined for Euler only");
    if (!(cfl > 0)) return fail(SWEPT_EINVAL, "cfl must be positive");
    *q = *prob;
    if (!(q->dt > 0)) q->dt = 1.0;  // dt is the output here; any positive value passes validation
    return derive(q, nullptr, d);
}

// The reduction itself: kParts partial maxima, then one fixed-order combine.
static int cfl_run(const swept_problem& q, const Derived& d, const void* d_state, double cfl, double* partials,
                   double* red, hipStream_t st, double* dt_out)
{
    const size_t NN = (size_t)q.nx * q.ny;
    hipError_t e = swept::launch_cfl_max(q.dtype, d_state, NN, q.gamma, d.dx, d.dy, partials, kParts, red, st);
    if (e != hipSuccess) return hip_fail(e, "cfl reduction");
    double smax = 0.0;
    e = hipMemcpyAsync(&smax, red, sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "cfl copy");
    if (!(smax > 0) || !std::isfinite(smax)) return fail(SWEPT_ENONFINITE, "max signal rate %g", smax);
    *dt_out = cfl / smax;
    return SWEPT_OK;
}

int swept_cfl_dt(const swept_problem* prob, const void* d_state, double cfl, void* d_work, size_t work_bytes,
                 void* hip_stream, double* dt_out)
{
    if (!d_work) return fail(SWEPT_EINVAL, "NULL argument");
    swept_problem q;
    Derived d;
    const int rc = cfl_check(prob, d_state, cfl, dt_out, &q, &d);
    if (rc) return rc;
    const size_t need = workspace_for(d);
    if (work_bytes < need) return fail(SWEPT_EWORKSPACE, "workspace %zu bytes < %zu needed", work_bytes, need);
    char* w = static_cast<char*>(d_work);
    double* partials = reinterpret_cast<double*>(w + align_up(d.state_bytes));
    double* red = reinterpret_cast<double*>(w + align_up(d.state_bytes) + align_up(sizeof(double) * 4 * kParts));
    return cfl_run(q, d, d_state, cfl, partials, red, reinterpret_cast<hipStream_t>(hip_stream), dt_out);
}

int swept_cfl_dt_noalloc(const swept_problem* prob, const void* d_state, double cfl, void* hip_stream,
                         double* dt_out)
{
    static_assert(swept::kNoAllocParts == kParts, "the static scratch holds exactly the reduction's partials");
    swept_problem q;
    Derived d;
    const int rc = cfl_check(prob, d_state, cfl, dt_out, &q, &d);  // rejects nx > 32768 (the scratch's limit)
    if (rc) return rc;
    double* scratch = nullptr;
    const hipError_t e = swept::noalloc_scratch(&scratch);
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    return cfl_run(q, d, d_state, cfl, scratch, scratch + kParts, reinterpret_cast<hipStream_t>(hip_stream), dt_out);
}

int swept_destroy(swept_ctx* c)
{
    delete c;
    return SWEPT_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- batch

struct swept_batch {
    int count = 0, dtype = 0;
    hipStream_t stream = nullptr;
    std::vector<swept_problem> probs;
    std::vector<Derived> d;
    std::vector<void*> states, buf1s;
    swept::PhaseArgs* dev_args = nullptr;
    int* ctr = nullptr;
    size_t lds = 0;
    int grid = 0;
    int mode = SWEPT_BATCH_COOPERATIVE;
};

namespace {

struct BatchLayout {
    std::vector<size_t> buf1_off, tab_off;
    size_t args_off, ctr_off, total;
};

int batch_derive(const swept_problem* probs, const swept_tuning* tunes, int32_t count, std::vector<Derived>* d,
                 BatchLayout* lay)
{
    if (!probs) return fail(SWEPT_EINVAL, "problems is NULL");
    if (count < 1 || count > swept::kBatchMax)
        return fail(SWEPT_EINVAL, "count=%d outside [1, %d]", count, swept::kBatchMax);
    d->resize(count);
    lay->buf1_off.resize(count);
    lay->tab_off.resize(count);
    size_t off = 0;
    for (int q = 0; q < count; ++q) {
        if (probs[q].dtype != probs[0].dtype) return fail(SWEPT_EINVAL, "all problems of a batch share one dtype");
        if (probs[q].kind == SWEPT_EULER && probs[q].boundary != SWEPT_BC_PERIODIC)
            return fail(SWEPT_ENOTSUP, "problem %d: the batch runs Euler periodic only", q);
        swept_tuning t{tunes ? tunes[q].tile : 0, swept::batch_wg(probs[0].dtype)};
        const int rc = derive(&probs[q], &t, &(*d)[q]);
        if (rc) return rc;
        lay->buf1_off[q] = off;
        off += align_up((*d)[q].state_bytes);
        lay->tab_off[q] = off;
        off += align_up(table_bytes((*d)[q]));
    }
    lay->args_off = off;
    lay->ctr_off = off + align_up(sizeof(swept::PhaseArgs) * count);
    lay->total = lay->ctr_off + align_up(2 * sizeof(int));
    return SWEPT_OK;
}

}  // namespace

extern "C" {

int swept_batch_workspace_bytes(const swept_problem* probs, const swept_tuning* tunes, int32_t count, size_t* bytes)
{
    if (!bytes) return fail(SWEPT_EINVAL, "bytes is NULL");
    std::vector<Derived> d;
    BatchLayout lay;
    const int rc = batch_derive(probs, tunes, count, &d, &lay);
    if (rc) return rc;
    *bytes = lay.total;
    return SWEPT_OK;
}

int swept_batch_init(swept_batch** ctx, const swept_problem* probs, const swept_tuning* tunes, void* const* d_states,
                     int32_t count, void* d_work, size_t work_bytes, void* hip_stream)
{
    if (!ctx) return fail(SWEPT_EINVAL, "ctx is NULL");
    *ctx = nullptr;
    std::vector<Derived> d;
    BatchLayout lay;
    int rc = batch_derive(probs, tunes, count, &d, &lay);
    if (rc) return rc;
    if (!d_states || !d_work) return fail(SWEPT_EINVAL, "NULL state array or workspace");
    for (int q = 0; q < count; ++q)
        if (!d_states[q] || reinterpret_cast<uintptr_t>(d_states[q]) % 16)
            return fail(SWEPT_EINVAL, "state %d is NULL or not 16-byte aligned", q);
    if (reinterpret_cast<uintptr_t>(d_work) % 16) return fail(SWEPT_EINVAL, "workspace not 16-byte aligned");
    if (work_bytes < lay.total) return fail(SWEPT_EWORKSPACE, "workspace %zu bytes < %zu needed", work_bytes, lay.total);
    swept_batch* b = new (std::nothrow) swept_batch();
    if (!b) return fail(SWEPT_EINVAL, "out of host memory");
    b->count = count;
    b->dtype = probs[0].dtype;
    b->stream = reinterpret_cast<hipStream_t>(hip_stream);
    b->probs.assign(probs, probs + count);
    b->d = d;
    char* w = static_cast<char*>(d_work);
    std::vector<swept::PhaseArgs> args(count);
    std::vector<std::vector<swept::LevelEntry>> tabs(count);
    for (int q = 0; q < count; ++q) {
        b->states.push_back(d_states[q]);
        b->buf1s.push_back(w + lay.buf1_off[q]);
        b->lds = std::max(b->lds, d[q].lds_bytes);
        tabs[q].resize(swept::level_table_entries(d[q].h));
        build_level_table(d[q], tabs[q].data());
        swept::PhaseArgs& a = args[q];
        a = swept::PhaseArgs{};
        a.buf0 = a.out0 = d_states[q];
        a.buf1 = a.out1 = w + lay.buf1_off[q];
        a.lvl0 = d_states[q];
        a.N = probs[q].nx;
        a.tile = d[q].tile;
        a.h = d[q].h;
        a.tiles = probs[q].nx / d[q].tile;
        a.kind = probs[q].kind;
        a.scheme = probs[q].scheme;
        a.bc = probs[q].boundary;
        a.tab = reinterpret_cast<swept::LevelEntry*>(w + lay.tab_off[q]);
        if (probs[q].kind == SWEPT_HEAT) {
            a.p[0] = d[q].r;
            a.p[1] = probs[q].boundary == SWEPT_BC_DIRICHLET ? probs[q].boundary_value : 0.0;
        } else {
            a.p[0] = probs[q].gamma;
            a.p[1] = 0.5 * probs[q].dt / d[q].dx;
            a.p[2] = 0.5 * probs[q].dt / d[q].dy;
            a.p[3] = probs[q].dt / d[q].dx;
            a.p[4] = probs[q].dt / d[q].dy;
        }
    }
    b->dev_args = reinterpret_cast<swept::PhaseArgs*>(w + lay.args_off);
    b->ctr = reinterpret_cast<int*>(w + lay.ctr_off);
    // the batch kernel also has a small static LDS array (its per-phase item prefix)
    const size_t dyn_max = kLdsMax - swept::kBatchStaticLds;
    if (b->lds > dyn_max) {
        delete b;
        return fail(SWEPT_ESHAPE, "batch needs %zu bytes of LDS per workgroup (max %zu)", b->lds, dyn_max);
    }
    hipError_t e = swept::set_batch_lds_limit(b->dtype, dyn_max);
    int bpc = 0, dev = 0, cus = 0;
    if (e == hipSuccess) e = swept::batch_occupancy(b->dtype, b->lds, &bpc);
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    for (int q = 0; q < count && e == hipSuccess; ++q)
        e = hipMemcpyAsync(w + lay.tab_off[q], tabs[q].data(), table_bytes(d[q]), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->dev_args, args.data(), sizeof(swept::PhaseArgs) * count, hipMemcpyHostToDevice,
                           b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
        delete b;
        return hip_fail(e, "batch init");
    }
    if (bpc < 1) {
        delete b;
        return fail(SWEPT_ESHAPE, "batch workgroup (%zu bytes of LDS) does not fit a compute unit", b->lds);
    }
    b->grid = bpc * cus;
    *ctx = b;
    return SWEPT_OK;
}

int swept_batch_advance(swept_batch* b, int64_t n_steps)
{
    if (!b) return fail(SWEPT_EINVAL, "ctx is NULL");
    if (n_steps < 0) return fail(SWEPT_EINVAL, "n_steps=%lld < 0", (long long)n_steps);
    if (n_steps == 0) return SWEPT_OK;
    if (n_steps > (int64_t)1 << 28) return fail(SWEPT_EINVAL, "n_steps too large");
    int nph = 0;
    for (int q = 0; q < b->count; ++q) {
        const int64_t L = n_steps * b->d[q].lps;
        nph = std::max(nph, (int)(2 * ((L + b->d[q].h - 1) / b->d[q].h) + 1));
    }
    hipError_t e = hipSuccess;
    if (b->mode == SWEPT_BATCH_COOPERATIVE) {
        e = swept::launch_batch(b->dtype, b->dev_args, b->count, nph, (long long)n_steps, b->grid, b->lds, b->stream,
                                b->ctr);
    } else {
        for (int gp = 0; gp < nph && e == hipSuccess; ++gp)
            e = swept::launch_batch_phase(b->dtype, b->dev_args, b->count, gp, (long long)n_steps, b->grid, b->lds,
                                          b->stream, b->ctr);
    }
    if (e != hipSuccess) return hip_fail(e, "batch launch");
    for (int q = 0; q < b->count; ++q) {
        if ((n_steps * b->d[q].lps) & 1) {
            e = hipMemcpyAsync(b->states[q], b->buf1s[q], b->d[q].state_bytes, hipMemcpyDeviceToDevice, b->stream);
            if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
        }
    }
    return SWEPT_OK;
}

int swept_batch_set_mode(swept_batch* b, int32_t mode)
{
    if (!b) return fail(SWEPT_EINVAL, "ctx is NULL");
    if (mode != SWEPT_BATCH_COOPERATIVE && mode != SWEPT_BATCH_PER_PHASE)
        return fail(SWEPT_EINVAL, "batch mode %d is neither cooperative (0) nor per phase (1)", (int)mode);
    b->mode = mode;
    return SWEPT_OK;
}

int swept_batch_query(const swept_batch* b, int32_t q, swept_info* info)
{
    if (!b || !info || q < 0 || q >= b->count) return fail(SWEPT_EINVAL, "bad argument");
    const Derived& d = b->d[q];
    info->nvar = d.nvar;
    info->n = d.n;
    info->levels_per_step = d.lps;
    info->tile = d.tile;
    info->h = d.h;
    info->wg = d.wg;
    info->r = d.r;
    info->dx = d.dx;
    info->dy = d.dy;
    info->state_bytes = d.state_bytes;
    info->lds_bytes = d.lds_bytes;
    return SWEPT_OK;
}

int swept_batch_grid(const swept_batch* b, int32_t* grid)
{
    if (!b || !grid) return fail(SWEPT_EINVAL, "bad argument");
    *grid = b->grid;
    return SWEPT_OK;
}

int swept_batch_set_stream(swept_batch* b, void* hip_stream)
{
    if (!b) return fail(SWEPT_EINVAL, "ctx is NULL");
    b->stream = reinterpret_cast<hipStream_t>(hip_stream);
    return SWEPT_OK;
}

int swept_batch_destroy(swept_batch* b)
{
    delete b;
    return SWEPT_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- heterogeneous share

struct swept_hetero {
    swept_ctx* ctx = nullptr;
    swept::Hetero* run = nullptr;
    int gpu_rows = 0, cpu_rows = 0, threads = 0;
};

extern "C" {

int swept_hetero_init(swept_hetero** out, swept_ctx* c, double gpu_share, int32_t cpu_threads)
{
    if (!out) return fail(SWEPT_EINVAL, "out is NULL");
    *out = nullptr;
    if (!c) return fail(SWEPT_EINVAL, "ctx is NULL");
    if (!(gpu_share >= 0.0 && gpu_share <= 1.0)) return fail(SWEPT_EINVAL, "gpu_share=%g outside [0, 1]", gpu_share);
    if (cpu_threads < 0 || cpu_threads > 1024) return fail(SWEPT_EINVAL, "cpu_threads=%d outside [0, 1024]", cpu_threads);
    if (c->prob.boundary != SWEPT_BC_PERIODIC)
        return fail(SWEPT_ENOTSUP, "the heterogeneous advance runs periodic problems only");
    const int tiles = c->prob.nx / c->d.tile;
    int threads = cpu_threads;
    if (threads == 0) {
        const char* env = std::getenv("OMP_NUM_THREADS");
        threads = env ? std::atoi(env) : 0;
        if (threads <= 0) threads = (int)std::thread::hardware_concurrency();
        if (threads <= 0) threads = 1;
        threads = std::min(threads, 256);
    }
    swept_hetero* h = new (std::nothrow) swept_hetero();
    if (!h) return fail(SWEPT_EINVAL, "out of host memory");
    h->ctx = c;
    h->gpu_rows = (int)std::floor(gpu_share * tiles + 0.5);  // Eq. 2: G = s W, in whole tile rows
    h->cpu_rows = tiles - h->gpu_rows;
    h->threads = threads;
    swept::HeteroSetup s;
    s.kind = c->prob.kind;
    s.dtype = c->prob.dtype;
    s.scheme = c->prob.scheme;
    s.N = c->prob.nx;
    s.b = c->d.tile;
    s.h = c->d.h;
    s.tiles = tiles;
    s.nvar = c->d.nvar;
    s.lps = c->d.lps;
    s.wg = c->d.wg;
    s.lds = c->d.lds_bytes;
    s.state_bytes = c->d.state_bytes;
    try {
        s.tab.resize(swept::level_table_entries(c->d.h));
    } catch (...) {
        delete h;
        return fail(SWEPT_EINVAL, "out of host memory");
    }
    build_level_table(c->d, s.tab.data());
    s.base = phase_args(c, 0);
    s.d0 = c->state;
    s.d1 = c->buf1;
    s.stream = c->stream;
    s.gpu_rows = h->gpu_rows;
    s.threads = threads;
    const hipError_t e = swept::hetero_create(s, &h->run);
    if (e != hipSuccess) {
        delete h;
        return hip_fail(e, "heterogeneous runner (pinned host buffers)");
    }
    *out = h;
    return SWEPT_OK;
}

int swept_hetero_advance(swept_hetero* h, int64_t n_steps)
{
    if (!h) return fail(SWEPT_EINVAL, "ctx is NULL");
    if (n_steps < 0) return fail(SWEPT_EINVAL, "n_steps=%lld < 0", (long long)n_steps);
    if (n_steps * h->ctx->d.lps > (int64_t)1 << 30) return fail(SWEPT_EINVAL, "n_steps too large");
    if (n_steps == 0) return SWEPT_OK;
    if (h->cpu_rows == 0) {  // share 1: the all-GPU advance
        const int rc = advance_impl(h->ctx, n_steps);
        if (rc) return rc;
        const hipError_t e = hipStreamSynchronize(h->ctx->stream);
        return e == hipSuccess ? SWEPT_OK : hip_fail(e, "hipStreamSynchronize");
    }
    const hipError_t e = swept::hetero_advance(h->run, (long long)n_steps, h->ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "heterogeneous advance");
    return SWEPT_OK;
}

int swept_hetero_query(const swept_hetero* h, int32_t* gpu_rows, int32_t* cpu_rows, int32_t* threads)
{
    if (!h || !gpu_rows || !cpu_rows || !threads) return fail(SWEPT_EINVAL, "NULL argument");
    *gpu_rows = h->gpu_rows;
    *cpu_rows = h->cpu_rows;
    *threads = h->threads;
    return SWEPT_OK;
}

int swept_hetero_destroy(swept_hetero* h)
{
    if (h) swept::hetero_destroy(h->run);
    delete h;
    return SWEPT_OK;
}

}  // extern "C"
