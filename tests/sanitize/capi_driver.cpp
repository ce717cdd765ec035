// Drives the argument validation of every C ABI entry point with invalid and
// valid arguments that never reach the HIP runtime, for the address and
// undefined-behaviour sanitizer build of tests/test_sanitizers.py.  Exits
// non-zero if a call returns an unexpected code.
#include <stdio.h>
#include <string.h>

#include "../../include/swept.h"

static int failures = 0;

static void expect(int got, int want, const char* what)
{
    if (got != want) {
        fprintf(stderr, "%s: got %d, want %d (%s)\n", what, got, want, swept_last_error());
        ++failures;
    }
}

static swept_problem heat(int n, double dt)
{
    swept_problem p;
    memset(&p, 0, sizeof p);
    p.kind = SWEPT_HEAT;
    p.dtype = SWEPT_F64;
    p.nx = p.ny = n;
    p.lx = p.ly = 1.0;
    p.dt = dt;
    p.alpha = 1.0;
    p.gamma = 1.4;
    return p;
}

static swept_problem euler(int n)
{
    swept_problem p = heat(n, 1e-3);
    p.kind = SWEPT_EULER;
    p.lx = p.ly = 10.0;
    return p;
}

int main(void)
{
    size_t bytes = 0;
    swept_tuning t = {0, 0};
    swept_problem p = heat(64, 0.2 / 64 / 64);
    expect(swept_workspace_bytes(&p, &t, &bytes), SWEPT_OK, "heat workspace");
    expect(swept_workspace_bytes(NULL, &t, &bytes), SWEPT_EINVAL, "null problem");
    expect(swept_workspace_bytes(&p, &t, NULL), SWEPT_EINVAL, "null bytes");
    swept_problem q = p;
    q.kind = 7;
    expect(swept_workspace_bytes(&q, &t, &bytes), SWEPT_EINVAL, "bad kind");
    q = p, q.dtype = 9;
    expect(swept_workspace_bytes(&q, &t, &bytes), SWEPT_EINVAL, "bad dtype");
    q = p, q.nx = q.ny = 0;
    expect(swept_workspace_bytes(&q, &t, &bytes), SWEPT_ESHAPE, "empty grid");
    q = p, q.ny = 32;
    expect(swept_workspace_bytes(&q, &t, &bytes), SWEPT_ESHAPE, "not square");
    q = p, q.nx = q.ny = 65536;
    expect(swept_workspace_bytes(&q, &t, &bytes), SWEPT_ESHAPE, "too large");
    q = p, q.dt = 1.0;
    expect(swept_workspace_bytes(&q, &t, &bytes), SWEPT_EUNSTABLE, "4r > 1");
    q = p, q.dt = -1.0;
    expect(swept_workspace_bytes(&q, &t, &bytes), SWEPT_EUNSTABLE, "dt < 0");
    q = p, q.boundary = 9;
    expect(swept_workspace_bytes(&q, &t, &bytes), SWEPT_EINVAL, "bad boundary");
    q = p, q.boundary = SWEPT_BC_REFLECT;
    expect(swept_workspace_bytes(&q, &t, &bytes), SWEPT_EINVAL, "heat slip wall");
    q = p, q.scheme = 1;
    expect(swept_workspace_bytes(&q, &t, &bytes), SWEPT_EINVAL, "heat scheme bits");
    swept_tuning bt = {12, 0};
    expect(swept_workspace_bytes(&p, &bt, &bytes), SWEPT_ESHAPE, "tile not dividing");
    bt.tile = 64;
    expect(swept_workspace_bytes(&p, &bt, &bytes), SWEPT_ESHAPE, "nx < 2 tile");
    bt.tile = 16, bt.wg = 100;
    expect(swept_workspace_bytes(&p, &bt, &bytes), SWEPT_EINVAL, "wg not a multiple of 64");
    swept_problem e = euler(64);
    expect(swept_workspace_bytes(&e, NULL, &bytes), SWEPT_OK, "euler workspace");
    swept_problem f = e;
    f.gamma = 1.0;
    expect(swept_workspace_bytes(&f, NULL, &bytes), SWEPT_EINVAL, "gamma 1");
    f = e, f.boundary = SWEPT_BC_DIRICHLET;
    expect(swept_workspace_bytes(&f, NULL, &bytes), SWEPT_ENOTSUP, "euler dirichlet");
    f = e, f.scheme = 8;
    expect(swept_workspace_bytes(&f, NULL, &bytes), SWEPT_EINVAL, "unknown scheme bit");
    for (int s = 0; s < 4; ++s)
        for (int bc = 0; bc < 4; bc += (bc == 0 ? 2 : 1)) {
            f = e, f.scheme = s, f.boundary = bc, f.dtype = s & 1;
            expect(swept_workspace_bytes(&f, NULL, &bytes), SWEPT_OK, "euler variants");
        }

    swept_ctx* ctx = (swept_ctx*)&bytes;
    alignas(16) static char fake[64];
    expect(swept_init(NULL, &p, &t, fake, fake, 1 << 20, NULL), SWEPT_EINVAL, "init null ctx");
    expect(swept_init(&ctx, &p, &t, NULL, fake, 1 << 20, NULL), SWEPT_EINVAL, "init null state");
    expect(swept_init(&ctx, &p, &t, fake, NULL, 1 << 20, NULL), SWEPT_EINVAL, "init null work");
    expect(swept_init(&ctx, &p, &t, fake + 1, fake, 1 << 20, NULL), SWEPT_EINVAL, "init misaligned");
    expect(swept_init(&ctx, &p, &t, fake, fake, 8, NULL), SWEPT_EWORKSPACE, "init small workspace");
    expect(swept_query(NULL, NULL), SWEPT_EINVAL, "query");
    expect(swept_set_stream(NULL, NULL), SWEPT_EINVAL, "set stream");
    expect(swept_advance(NULL, 1), SWEPT_EINVAL, "advance");
    expect(standard_advance(NULL, 1), SWEPT_EINVAL, "standard");
    expect(swept_conserved(NULL, NULL), SWEPT_EINVAL, "conserved");
    expect(swept_tape_bytes(NULL, 1, &bytes), SWEPT_EINVAL, "tape bytes");
    expect(swept_adjoint(NULL, 1, NULL, 0, NULL, NULL, NULL), SWEPT_EINVAL, "adjoint");
    double dt = 0;
    expect(swept_cfl_dt(&p, fake, 0.4, fake, 1 << 30, NULL, &dt), SWEPT_ENOTSUP, "cfl heat");
    expect(swept_cfl_dt(&e, fake, 0.4, NULL, 1 << 30, NULL, &dt), SWEPT_EINVAL, "cfl null work");
    expect(swept_cfl_dt(&e, fake, -1.0, fake, 1 << 30, NULL, &dt), SWEPT_EINVAL, "cfl negative");
    expect(swept_cfl_dt(&e, fake, 0.4, fake, 8, NULL, &dt), SWEPT_EWORKSPACE, "cfl small workspace");
    swept_problem big = euler(65536);
    expect(swept_cfl_dt_noalloc(&big, fake, 0.4, NULL, &dt), SWEPT_ESHAPE, "noalloc oversized");
    expect(swept_cfl_dt_noalloc(NULL, fake, 0.4, NULL, &dt), SWEPT_EINVAL, "noalloc null");

    swept_problem probs[3] = {heat(128, 0.2 / 128 / 128), euler(64), heat(256, 0.1 / 256 / 256)};
    expect(swept_batch_workspace_bytes(probs, NULL, 3, &bytes), SWEPT_OK, "batch workspace");
    expect(swept_batch_workspace_bytes(probs, NULL, 0, &bytes), SWEPT_EINVAL, "batch empty");
    expect(swept_batch_workspace_bytes(NULL, NULL, 3, &bytes), SWEPT_EINVAL, "batch null");
    probs[1].dtype = SWEPT_F32;
    expect(swept_batch_workspace_bytes(probs, NULL, 3, &bytes), SWEPT_EINVAL, "batch mixed dtypes");
    probs[1].dtype = SWEPT_F64, probs[1].boundary = SWEPT_BC_REFLECT;
    expect(swept_batch_workspace_bytes(probs, NULL, 3, &bytes), SWEPT_ENOTSUP, "batch euler walls");
    probs[1].boundary = 0;
    swept_batch* bctx = NULL;
    expect(swept_batch_init(&bctx, probs, NULL, NULL, 3, fake, 1 << 20, NULL), SWEPT_EINVAL, "batch null states");
    expect(swept_batch_advance(NULL, 1), SWEPT_EINVAL, "batch advance");
    expect(swept_batch_set_mode(NULL, 0), SWEPT_EINVAL, "batch mode");
    int32_t g = 0, c = 0, th = 0;
    expect(swept_batch_grid(NULL, &g), SWEPT_EINVAL, "batch grid");

    swept_hetero* h = NULL;
    expect(swept_hetero_init(&h, NULL, 0.5, 0), SWEPT_EINVAL, "hetero null ctx");
    expect(swept_hetero_init(NULL, NULL, 0.5, 0), SWEPT_EINVAL, "hetero null out");
    expect(swept_hetero_advance(NULL, 1), SWEPT_EINVAL, "hetero advance");
    expect(swept_hetero_query(NULL, &g, &c, &th), SWEPT_EINVAL, "hetero query");

    expect(swept_destroy(NULL), SWEPT_OK, "destroy null");
    expect(swept_batch_destroy(NULL), SWEPT_OK, "batch destroy null");
    expect(swept_hetero_destroy(NULL), SWEPT_OK, "hetero destroy null");
    printf("capi validation: %d failures\n", failures);
    return failures ? 1 : 0;
}
