/*
 * oracle_abi.c -- the CPU oracle behind the same C entry points as the GPU
 * library (lb_init, lb_step, lb_moments, lb_pseudo_energy, lb_trace, ...),
 * on host memory.
 *
 * TEST INFRASTRUCTURE ONLY, like oracle.c: it lets the tests and the
 * benchmark's CPU-baseline leg drive the oracle through the same sequence of
 * calls as the GPU library.  It shares no source with the HIP library: the
 * parameter block below is this file's own declaration of the interface's
 * layout (the interface has to match; the code does not).
 *
 * Semantics follow the interface: the state is the pre-collision
 * populations at time t (t = 0 the initial equilibrium), a call that fails
 * changes nothing, and with log_every > 0 the section V observables of every
 * log point t' in [t, t+n) are recorded by lb_step before the step that
 * leaves t' (lb_trace records the current t if it is a log point).
 * Differences: every pointer is host memory (on_device must be 0), the
 * storage must match the library's arithmetic (LB_F64 for liboracle.so,
 * LB_F32 for the single-precision twin), and the "workspace" is a host
 * buffer holding the populations and the trace.
 */
#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#ifdef ORACLE_F32
typedef float real;
#define ORACLE_STORAGE 1
#else
typedef double real;
#define ORACLE_STORAGE 0
#endif

/* Entry points of oracle.c. */
void orc_tables(int8_t cx[24], int8_t cy[24], double K[24], double KE[25], double G1, double G2);
void orc_init(int64_t nx, int64_t ny, const double* rho, const double* ux, const double* uy, real* f);
void orc_moments(int64_t nx, int64_t ny, const real* f, real* rho, real* jx, real* jy);
int orc_step(int64_t nx, int64_t ny, double tau, double rho0, double G1, double G2, real* f,
             int64_t nsteps);
int orc_observables(int64_t nx, int64_t ny, double rho0, double G1, double G2, const real* f,
                    double out[5]);

enum { OK = 0, ERR_INVALID = -1, ERR_HIP = -2, ERR_NONFINITE = -3, ERR_STATE = -4 };

/* Layout of the interface's parameter block. */
typedef struct {
    int32_t nx, ny, storage, log_every, tile_x, tile_y, tile_rows, steps_per_launch;
    int64_t trace_cap;
    double tau, rho0, G1, G2, rho_ref;
} params;

typedef struct lb_ctx {
    params p;
    real* f;         /* 9 * nx * ny, in the caller's workspace */
    double* trace;   /* trace_cap * 6, in the caller's workspace */
    int64_t t, rows, last_logged;
} lb_ctx;

static _Thread_local char g_err[512];

static int fail(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

static int check(const params* p)
{
    if (!p) return fail(ERR_INVALID, "params is NULL");
    if (p->nx < 5 || p->ny < 5) return fail(ERR_INVALID, "nx, ny must be >= 5");
    if (p->storage != ORACLE_STORAGE)
        return fail(ERR_INVALID, "this oracle library computes with storage %d only", ORACLE_STORAGE);
    if (p->log_every < 0 || p->trace_cap < 0) return fail(ERR_INVALID, "negative log_every or trace_cap");
    if (p->steps_per_launch < 0 || p->steps_per_launch > 2)
        return fail(ERR_INVALID, "steps_per_launch must be 0, 1 or 2");
    if (!isfinite(p->tau) || !(p->tau > 0.5)) return fail(ERR_INVALID, "tau must be finite and > 0.5");
    if (!isfinite(p->rho0) || !(p->rho0 > 0.0)) return fail(ERR_INVALID, "rho0 must be finite and > 0");
    if (!isfinite(p->G1) || !isfinite(p->G2)) return fail(ERR_INVALID, "G1, G2 must be finite");
    return OK;
}

static size_t pop_bytes(const params* p)
{
    size_t b = (size_t)9 * (size_t)p->nx * (size_t)p->ny * sizeof(real);
    return (b + 255) / 256 * 256;
}

static int record(lb_ctx* c)
{
    double o[5];
    if (orc_observables(c->p.nx, c->p.ny, c->p.rho0, c->p.G1, c->p.G2, c->f, o))
        return fail(ERR_INVALID, "out of host memory");
    double* row = c->trace + c->rows * 6;
    row[0] = (double)c->t;
    for (int k = 0; k < 5; ++k) row[1 + k] = o[k];
    c->last_logged = c->t;
    ++c->rows;
    return OK;
}

const char* lb_last_error(void) { return g_err; }

int lb_validate(const params* p) { return check(p); }

static size_t ws_bytes(const params* p)
{
    return pop_bytes(p) + (size_t)p->trace_cap * 6 * sizeof(double);
}

size_t lb_workspace_bytes(const params* p)
{
    return check(p) ? 0 : ws_bytes(p);
}

/* The oracle has no tiles: one pass covers the lattice. */
int lb_launch_shape(const params* p, int32_t* tile_x, int32_t* tile_y, int32_t* tile_rows,
                    int32_t* blocks)
{
    int rc = check(p);
    if (rc) return rc;
    if (tile_x) *tile_x = p->nx;
    if (tile_y) *tile_y = p->ny;
    if (tile_rows) *tile_rows = 1;
    if (blocks) *blocks = 1;
    return OK;
}

/* Nor launches: no step is fused with another. */
int lb_two_step_shape(const params* p, int32_t* tile_x, int32_t* tile_y, int32_t* blocks)
{
    int rc = check(p);
    if (rc) return rc;
    if (tile_x) *tile_x = 0;
    if (tile_y) *tile_y = 0;
    if (blocks) *blocks = 0;
    return OK;
}

int lb_tables(const params* p, int8_t cx[24], int8_t cy[24], double K[24], double KE[25])
{
    int rc = check(p);
    if (rc) return rc;
    if (!cx || !cy || !K || !KE) return fail(ERR_INVALID, "NULL output");
    orc_tables(cx, cy, K, KE, p->G1, p->G2);
    return OK;
}

int lb_init(lb_ctx** out, const params* p, void* workspace, size_t bytes, const double* rho,
            const double* ux, const double* uy, int on_device, void* stream)
{
    (void)stream;
    if (!out) return fail(ERR_INVALID, "out is NULL");
    *out = NULL;
    int rc = check(p);
    if (rc) return rc;
    if (on_device) return fail(ERR_INVALID, "the oracle takes host memory only");
    if (!workspace || !rho) return fail(ERR_INVALID, "NULL workspace or rho_init");
    if (bytes < ws_bytes(p)) return fail(ERR_INVALID, "workspace too small");
    const int64_t N = (int64_t)p->nx * p->ny;
    for (int64_t s = 0; s < N; ++s) {
        if (!isfinite(rho[s]) || !(rho[s] > 0.0)) return fail(ERR_INVALID, "rho_init[%lld] invalid", (long long)s);
        if ((ux && !isfinite(ux[s])) || (uy && !isfinite(uy[s])))
            return fail(ERR_INVALID, "u_init[%lld] is not finite", (long long)s);
    }
    lb_ctx* c = (lb_ctx*)calloc(1, sizeof *c);
    if (!c) return fail(ERR_INVALID, "out of host memory");
    c->p = *p;
    c->f = (real*)workspace;
    c->trace = (double*)((char*)workspace + pop_bytes(p));
    c->t = 0;
    c->rows = 0;
    c->last_logged = -1;
    orc_init(p->nx, p->ny, rho, ux, uy, c->f);
    *out = c;
    return OK;
}

int lb_step(lb_ctx* c, int64_t n)
{
    if (!c) return fail(ERR_STATE, "unknown context");
    if (n < 0) return fail(ERR_INVALID, "n must be >= 0");
    const int64_t le = c->p.log_every;
    int64_t need = 0;
    if (le > 0)
        for (int64_t t = c->t; t < c->t + n; ++t)
            if (t % le == 0 && t != c->last_logged) ++need;
    if (c->rows + need > c->p.trace_cap) return fail(ERR_STATE, "trace full");
    const int64_t end = c->t + n;
    while (c->t < end) {
        if (le > 0 && c->t % le == 0 && c->t != c->last_logged) {
            int rc = record(c);
            if (rc) return rc;
        }
        /* Advance to the next log point (or the end) in one call. */
        int64_t run = end - c->t;
        if (le > 0) {
            const int64_t to_log = le - c->t % le;
            if (to_log < run) run = to_log;
        }
        if (orc_step(c->p.nx, c->p.ny, c->p.tau, c->p.rho0, c->p.G1, c->p.G2, c->f, run))
            return fail(ERR_INVALID, "out of host memory");
        c->t += run;
    }
    return OK;
}

int lb_time(lb_ctx* c, int64_t* t)
{
    if (!c) return fail(ERR_STATE, "unknown context");
    if (!t) return fail(ERR_INVALID, "t is NULL");
    *t = c->t;
    return OK;
}

int lb_moments(lb_ctx* c, double* rho, double* ux, double* uy, int on_device)
{
    if (!c) return fail(ERR_STATE, "unknown context");
    if (on_device) return fail(ERR_INVALID, "the oracle takes host memory only");
    const int64_t N = (int64_t)c->p.nx * c->p.ny;
    real* m = (real*)malloc(sizeof(real) * 3 * N);
    if (!m) return fail(ERR_INVALID, "out of host memory");
    orc_moments(c->p.nx, c->p.ny, c->f, m, m + N, m + 2 * N);
    for (int64_t s = 0; s < N; ++s) {
        if (rho) rho[s] = (double)m[s];
        if (ux) ux[s] = (double)m[N + s] / (double)m[s];
        if (uy) uy[s] = (double)m[2 * N + s] / (double)m[s];
    }
    free(m);
    return OK;
}

int lb_pseudo_energy(lb_ctx* c, double out[6])
{
    if (!c) return fail(ERR_STATE, "unknown context");
    if (!out) return fail(ERR_INVALID, "out is NULL");
    double o[5];
    if (orc_observables(c->p.nx, c->p.ny, c->p.rho0, c->p.G1, c->p.G2, c->f, o))
        return fail(ERR_INVALID, "out of host memory");
    out[0] = (double)c->t;
    for (int k = 0; k < 5; ++k) out[1 + k] = o[k];
    for (int k = 0; k < 6; ++k)
        if (!isfinite(out[k])) return fail(ERR_NONFINITE, "non-finite mass or energy");
    return OK;
}

int lb_trace(lb_ctx* c, double* out, int64_t cap, int64_t* n_rows)
{
    if (!c) return fail(ERR_STATE, "unknown context");
    if (cap < 0 || (cap > 0 && !out)) return fail(ERR_INVALID, "bad output buffer");
    const int64_t le = c->p.log_every;
    if (le > 0 && c->t % le == 0 && c->t != c->last_logged && c->rows < c->p.trace_cap) {
        int rc = record(c);
        if (rc) return rc;
    }
    const int64_t rows = cap < c->rows ? cap : c->rows;
    if (rows > 0) memcpy(out, c->trace, (size_t)rows * 6 * sizeof(double));
    if (n_rows) *n_rows = c->rows;
    for (int64_t k = 0; k < rows * 6; ++k)
        if (!isfinite(out[k])) return fail(ERR_NONFINITE, "non-finite value in the trace");
    return OK;
}

int lb_get_state(lb_ctx* c, void* dst, int on_device)
{
    if (!c) return fail(ERR_STATE, "unknown context");
    if (on_device) return fail(ERR_INVALID, "the oracle takes host memory only");
    if (!dst) return fail(ERR_INVALID, "dst is NULL");
    memcpy(dst, c->f, (size_t)9 * c->p.nx * c->p.ny * sizeof(real));
    return OK;
}

int lb_set_state(lb_ctx* c, const void* src, int on_device, int64_t t)
{
    if (!c) return fail(ERR_STATE, "unknown context");
    if (on_device) return fail(ERR_INVALID, "the oracle takes host memory only");
    if (!src) return fail(ERR_INVALID, "src is NULL");
    if (t < 0) return fail(ERR_INVALID, "t must be >= 0");
    memcpy(c->f, src, (size_t)9 * c->p.nx * c->p.ny * sizeof(real));
    c->t = t;
    c->last_logged = -1;
    return OK;
}

int lb_destroy(lb_ctx* c)
{
    if (!c) return fail(ERR_STATE, "unknown context");
    free(c);
    return OK;
}
