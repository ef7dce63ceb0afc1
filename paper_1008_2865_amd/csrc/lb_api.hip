// Host side of liblb.so: the C ABI declared in include/lb.h.
//
// Validates every argument on the host before any launch, carves the
// caller's device workspace, keeps the time step, the ping-pong buffer
// index and the trace bookkeeping, and issues the kernels of
// lb_kernels.hip on the caller's stream.
#include "lb.h"
#include "lb_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <set>
#include <utility>
#include <string>
#include <vector>

using lbk::Coef;
using lbk::Geom;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what)
{
    return fail(LB_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Table 1 weights p(|c|^2), the D2Q9 weights w and the first-belt rest
// weight p_s0 = 1 - sum_k p_k = 247/420 implied by eq. (weights_1).
constexpr double kP1 = 4.0 / 63.0, kP2 = 4.0 / 135.0, kP4 = 1.0 / 180.0,
                 kP5 = 2.0 / 945.0, kP8 = 1.0 / 15120.0;
constexpr double kW0 = 4.0 / 9.0, kW1 = 1.0 / 9.0, kW2 = 1.0 / 36.0;
constexpr double kPS0 = 247.0 / 420.0;

// Link order: first belt in D2Q9 order, then |c|^2 = 4, 5, 8, each
// counter-clockwise from +x.
constexpr int kLX[24] = {1, 0, -1, 0, 1, -1, -1, 1, 2, 0, -2, 0,
                         2, 1, -1, -2, -2, -1, 1, 2, 2, -2, -2, 2};
constexpr int kLY[24] = {0, 1, 0, -1, 1, 1, -1, -1, 0, 2, 0, -2,
                         1, 2, 2, 1, -1, -2, -2, -1, 2, 2, -2, -2};

double coupling(int k, double G1, double G2)
{
    const int c2 = kLX[k] * kLX[k] + kLY[k] * kLY[k];
    const double p = c2 == 1 ? kP1 : c2 == 2 ? kP2 : c2 == 4 ? kP4 : c2 == 5 ? kP5 : kP8;
    if (k < 8) return G1 * (c2 == 1 ? kW1 : kW2) + G2 * p;
    return G2 * p;
}

Coef make_coef(const lb_params& p)
{
    Coef c;
    c.K1 = coupling(0, p.G1, p.G2);
    c.K2 = coupling(4, p.G1, p.G2);
    c.K4 = coupling(8, p.G1, p.G2);
    c.K5 = coupling(12, p.G1, p.G2);
    c.K8 = coupling(20, p.G1, p.G2);
    c.KE0 = p.G1 * kW0 + p.G2 * kPS0;
    c.tau = p.tau;
    c.omega = 1.0 / p.tau;
    c.sqrt_rho0 = std::sqrt(p.rho0);
    c.inv_rho0 = 1.0 / p.rho0;
    c.rho_ref = p.storage == LB_F16DEV ? p.rho_ref : 0.0;
    c.step = 0;
    return c;
}

int check_params(const lb_params* p)
{
    if (!p) return fail(LB_ERR_INVALID, "params is NULL");
    if (p->nx < 5 || p->ny < 5)
        return fail(LB_ERR_INVALID, "nx, ny must be >= 5 (got %d x %d)", p->nx, p->ny);
    // One population plane, padded rows included, must be indexable with
    // 32-bit offsets.
    if (((int64_t)p->nx + 192) * p->ny >= (int64_t(1) << 31))
        return fail(LB_ERR_INVALID, "(nx + 192) * ny must be < 2^31");
    // The moments, initialisation and state kernels put rows on the grid's
    // second dimension.
    if (p->ny > 65535) return fail(LB_ERR_INVALID, "ny must be <= 65535 (got %d)", p->ny);
    if (p->storage != LB_F64 && p->storage != LB_F32 && p->storage != LB_F16DEV)
        return fail(LB_ERR_INVALID, "unknown storage %d", p->storage);
    if (p->log_every < 0) return fail(LB_ERR_INVALID, "log_every must be >= 0");
    if (p->trace_cap < 0) return fail(LB_ERR_INVALID, "trace_cap must be >= 0");
    if (p->tile_x != 0 && p->tile_x != 64 && p->tile_x != 128 && p->tile_x != 256)
        return fail(LB_ERR_INVALID, "tile_x must be 0, 64, 128 or 256 (got %d)", p->tile_x);
    if (p->tile_y < 0 || p->tile_y > 4096)
        return fail(LB_ERR_INVALID, "tile_y must be in [0, 4096] (got %d)", p->tile_y);
    if (p->tile_rows < 0 || p->tile_rows > 2)
        return fail(LB_ERR_INVALID, "tile_rows must be 0, 1 or 2 (got %d)", p->tile_rows);
    if (p->steps_per_launch < 0 || p->steps_per_launch > 2)
        return fail(LB_ERR_INVALID, "steps_per_launch must be 0, 1 or 2 (got %d)", p->steps_per_launch);
    if (!std::isfinite(p->tau) || !(p->tau > 0.5))
        return fail(LB_ERR_INVALID, "tau must be finite and > 0.5");
    if (!std::isfinite(p->rho0) || !(p->rho0 > 0.0))
        return fail(LB_ERR_INVALID, "rho0 must be finite and > 0");
    if (!std::isfinite(p->G1) || !std::isfinite(p->G2))
        return fail(LB_ERR_INVALID, "G1, G2 must be finite");
    if (p->storage == LB_F16DEV && (!std::isfinite(p->rho_ref) || !(p->rho_ref > 0.0)))
        return fail(LB_ERR_INVALID, "rho_ref must be finite and > 0 for LB_F16DEV");
    return LB_OK;
}

// Launch shape and layout.  Defaults: the widest column strip (256, 128 or
// 64 columns) that the lattice fills, and the tallest tile of 32, 16, 8, 4
// or 2 rows that still gives at least 512 workgroups.
Geom make_geom(const lb_params& p)
{
    Geom g;
    g.nx = p.nx;
    g.ny = p.ny;
    // Row pitch: a multiple of 64 elements whose count of 64-element blocks
    // is odd, so consecutive rows (and the rows that concurrently running
    // workgroups touch) do not sit at power-of-two strides, which would
    // pile their accesses onto the same HBM channels.
    g.pitch = (p.nx + 63) / 64 * 64;
    if ((g.pitch / 64) % 2 == 0) g.pitch += 64;  // pitch <= nx + 127
    g.plane = (int64_t)p.ny * g.pitch;
    g.tile_x = p.tile_x ? p.tile_x : (p.nx >= 256 ? 256 : p.nx >= 128 ? 128 : 64);
    g.tiles_x = (p.nx + g.tile_x - 1) / g.tile_x;
    if (p.tile_y) {
        g.tile_y = p.tile_y;
    } else {
        // The tallest tile of 32, 16, 8, 4 or 2 rows that still gives at
        // least 512 workgroups (two per CU): tall tiles re-read fewer halo
        // rows, but a lattice of a few hundred rows would otherwise leave
        // most of the 256 CUs idle.
        g.tile_y = 32;
        while (g.tile_y > 2 && (int64_t)g.tiles_x * ((p.ny + g.tile_y - 1) / g.tile_y) < 512)
            g.tile_y /= 2;
    }
    if (g.tile_y > p.ny) g.tile_y = p.ny;
    g.rows_per_iter = p.tile_rows ? p.tile_rows : 1;
    g.blocks = g.tiles_x * ((p.ny + g.tile_y - 1) / g.tile_y);
    return g;
}

// Geometry of the two-step launches: tiles of tile_x lanes that produce
// tile_x - 6 columns (the first step also covers 3 columns each side).
// Explicit tile_x / tile_y apply to both kernels; the library's choice
// follows.
// Workgroups of the two-step kernel resident at once: the runtime's
// occupancy query on the current device (registers and LDS of the kernel as
// built) times its compute units.  Without a device to ask, the value for
// the MI355X as the kernel is built today: 3 waves per SIMD, i.e. 6
// workgroups of 128 lanes or 3 of 256 lanes per CU, on 256 CUs (a GPU test
// holds this to the occupancy query).
int64_t step2_slots_fallback(int tile_x) { return 256 * (tile_x == 256 ? 3 : 6); }
int64_t step2_slots(int storage, int tile_x)
{
    const int r = lbk::step2_resident(storage == LB_F16DEV ? LB_F16DEV : LB_F32, tile_x);
    return r > 0 ? r : step2_slots_fallback(tile_x);
}

// Two-step launch shape.  A workgroup walks its rows one after the other,
// so while every tile is resident at once (one round), shorter tiles finish
// sooner: the default takes the shortest tiles (128 lanes, else 256) that
// all fit in one round, up to 48 rows.  Past that, a launch of more than
// one round pays for a last round left partly empty, and a taller tile for
// fewer recomputed halo rows:
//   - single precision: 256-lane tiles filling one round when they are at
//     most 96 rows tall, else tiles of about 48 rows, a few rows shorter
//     when that fills the last round, or, when the last round would be
//     under half full, the height that fills one round fewer (at most 56);
//   - half storage, whose two-step kernel is not bound by memory: the
//     tallest 256-lane tiles of at most 128 rows whose last round is full.
// Measured on MI355X (FP32, us/step; one step per launch in brackets):
//   1200^2 128x8 18.0 (20.0);  1800^2 128x18 30.0, 128x24 33.3 (43.0);
//   2048^2 128x23 41.4, 128x24 42.1 (61.2);  2500^2 128x48 66.2, 128x40
//   66.7 (115.7);  3000^2 256x47 81.3, 256x48 83.0, 128x48 108.6 (151.9);
//   4096^2 256x92 144.0, 128x92 146.2, 256x46 147.5 (243.9);  5120^2
//   256x47 227.7, 256x71 231.5, 256x143 233.7;  8192^2 256x45 589.6,
//   256x48 604.6, 256x90 601.6, 256x179 619.7, 128x48 658.4 (1037.9).
// Half storage, us per launch: 8192^2 256x119 840-848 (three rounds),
// 256x90 847, 256x179 850, 256x357 860, 256x56 857-872 (6.3 rounds),
// 256x104 883 (3.4 rounds), 256x164 907 (2.1 rounds); 4096^2 256x92 235,
// 256x46 241-243, 256x56 248.
Geom make_geom2(const lb_params& p, const Geom& g)
{
    Geom g2 = g;
    auto strips = [&](int tx) { return (int64_t)(p.nx + tx - 7) / (tx - 6); };
    auto rows = [&](int ty) { return (int64_t)(p.ny + ty - 1) / ty; };
    // Height of the tiles of tx lanes that fill nr rounds (their count is at
    // most nr rounds' worth, and just under it).
    auto fill = [&](int tx, int64_t nr) -> int64_t {
        const int64_t per_strip = nr * step2_slots(p.storage, tx) / strips(tx);
        return per_strip > 0 ? (p.ny + per_strip - 1) / per_strip : (int64_t)p.ny;
    };
    int tx = p.tile_x, ty = p.tile_y;
    if (!tx || !ty) {
        int one_x = 0, one_y = 0;
        for (int c : {128, 256}) {
            if (tx && tx != c) continue;
            const int64_t per_strip = step2_slots(p.storage, c) / strips(c);
            if (per_strip < 1) continue;
            const int64_t h = (p.ny + per_strip - 1) / per_strip;
            if (h <= 48) {
                one_x = c;
                one_y = (int)h;
                break;
            }
        }
        if (one_x) {
            if (!tx) tx = one_x;
            if (!ty) ty = one_y;
        } else {
            if (!tx) tx = 256;
            if (!ty) {
                if (p.storage == LB_F16DEV) {
                    int64_t nr = 1;
                    while (fill(tx, nr) > 128) ++nr;
                    ty = (int)fill(tx, nr);
                } else if (fill(tx, 1) <= 96) {
                    ty = (int)fill(tx, 1);
                } else {
                    ty = 48;
                    const int64_t slots = step2_slots(p.storage, tx);
                    const int64_t tiles = strips(tx) * rows(48);
                    const int64_t rounds = (tiles + slots - 1) / slots;
                    const int64_t fit = fill(tx, rounds);
                    if (fit >= 44 && fit < 48)
                        ty = (int)fit;
                    else if (rounds > 1 && 2 * (tiles - (rounds - 1) * slots) < slots &&
                             fill(tx, rounds - 1) <= 56)
                        ty = (int)fill(tx, rounds - 1);
                }
            }
        }
    }
    g2.tile_x = tx;
    g2.tile_y = ty > p.ny ? p.ny : ty;
    const int w = g2.tile_x - 6;
    g2.tiles_x = (p.nx + w - 1) / w;
    g2.blocks = g2.tiles_x * ((p.ny + g2.tile_y - 1) / g2.tile_y);
    g2.rows_per_iter = 1;
    return g2;
}

// Whether plain steps run two per launch: FP32 or half storage when asked
// for (steps_per_launch = 2), and by default on lattices large enough for
// tiles of 8 rows or more (below that the one-step kernel is as fast or
// faster: FP32 1024^2 16.6 us/step either way, 512^2 11.7 against 7.7;
// half storage 1024^2 18.1 against 15.5).  Half storage, two per launch
// against one: 2048^2 41.1 against 48.1 us/step, 4096^2 152.8 against
// 166.3, 8192^2 551 against 627.
bool use_two(const lb_params& p, const Geom& g2)
{
    if (p.storage != LB_F32 && p.storage != LB_F16DEV) return false;
    if (p.steps_per_launch == 2) return true;
    return p.steps_per_launch == 0 && g2.tile_y >= 8;
}

// Workspace layout, each region 256-byte aligned.
struct Layout {
    size_t buf[2], partials, trace, scalars, staging, total;
};

Layout make_layout(const lb_params& p, const Geom& g)
{
    Layout L;
    const size_t pop = align_up((size_t)9 * g.plane * lbk::storage_bytes(p.storage));
    size_t off = 0;
    L.buf[0] = off; off += pop;
    L.buf[1] = off; off += pop;
    L.partials = off; off += align_up((size_t)g.blocks * 4 * sizeof(double));
    L.trace = off; off += align_up((size_t)p.trace_cap * 6 * sizeof(double));
    L.scalars = off; off += align_up(8 * sizeof(double));
    L.staging = off; off += align_up((size_t)3 * p.nx * p.ny * sizeof(double));
    L.total = off;
    return L;
}

}  // namespace

struct lb_ctx {
    lb_params p;
    Geom g;
    Geom g2;     // two-step launches: tile_x lanes make tile_x - 6 columns
    bool two;    // plain steps run two per launch where they can
    Coef coef;
    int device;
    hipStream_t stream;
    char* ws;
    void* buf[2];
    int cur;
    double* partials;
    double* trace;
    double* scalars;
    double* staging;
    int64_t t;
    int64_t trace_rows;
    int64_t last_logged;
    lb_batch* batch;  // non-NULL for a lattice owned by a batch
};

struct lb_batch {
    std::vector<lb_ctx*> members;
    lbk::BatchLattice* desc;   // device
    int32_t* tile_lattice;     // device
    int32_t* tile_lattice2;    // device, two-step tiles (when two)
    double* partials;          // device, 4 per tile
    int tiles, tiles2;
    bool two;                  // plain steps run two per launch
    int tile_x2, tile_y2;
    int storage, tile_x, rows_per_iter, min_tile_y;
    int device;
    hipStream_t stream;
    int parity;
    int64_t t, log_every, trace_cap, trace_rows, last_logged;
    bool use_graphs;
    std::map<std::pair<int64_t, int>, hipGraphExec_t> graphs;
    std::vector<lb_params> params;           // per lattice, as given to lb_batch_init
    std::vector<lbk::BatchLattice> host_desc;  // host copy of desc
    int tiles2_cap;                          // capacity of tile_lattice2
};

namespace {

std::mutex g_mu;
std::set<lb_ctx*> g_live;

int check_ctx(lb_ctx* c)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (!c || !g_live.count(c)) return fail(LB_ERR_STATE, "unknown or destroyed context");
    return LB_OK;
}

// Makes the context's device current for the duration of a call.
struct DeviceGuard {
    int prev = -1;
    hipError_t err = hipSuccess;
    explicit DeviceGuard(int dev)
    {
        err = hipGetDevice(&prev);
        if (err == hipSuccess && prev != dev) err = hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int now = -1;
        if (prev >= 0 && hipGetDevice(&now) == hipSuccess && now != prev) (void)hipSetDevice(prev);
    }
};

int field_check_host(const double* v, int64_t n, bool positive, const char* name)
{
    for (int64_t i = 0; i < n; ++i) {
        if (!std::isfinite(v[i]) || (positive && !(v[i] > 0.0)))
            return fail(LB_ERR_INVALID, "%s[%lld] = %g is not %s", name, (long long)i, v[i],
                        positive ? "finite and > 0" : "finite");
    }
    return LB_OK;
}

int energy_row(lb_ctx* c, int mode, const void* src, void* dst, double* row)
{
    c->coef.step = (uint32_t)c->t;
    hipError_t e = lbk::launch_step(c->p.storage, mode, src, dst, c->g, c->coef, c->partials, c->stream);
    if (e != hipSuccess) return hip_fail(e, "step kernel launch");
    e = lbk::launch_final(c->partials, c->g.blocks, (double)c->t, 0.5 * (c->p.G1 + c->p.G2), row,
                          c->stream);
    if (e != hipSuccess) return hip_fail(e, "final reduction launch");
    return LB_OK;
}

bool rows_finite(const double* r, int64_t n)
{
    for (int64_t i = 0; i < n * 6; ++i)
        if (!std::isfinite(r[i])) return false;
    return true;
}

}  // namespace

extern "C" {

const char* lb_last_error(void) { return g_err.c_str(); }

int lb_validate(const lb_params* p) { return check_params(p); }

size_t lb_workspace_bytes(const lb_params* p)
{
    if (check_params(p) != LB_OK) return 0;
    const Geom g = make_geom(*p);
    return make_layout(*p, g).total;
}

int lb_launch_shape(const lb_params* p, int32_t* tile_x, int32_t* tile_y, int32_t* tile_rows,
                    int32_t* blocks)
{
    int rc = check_params(p);
    if (rc) return rc;
    const Geom g = make_geom(*p);
    if (tile_x) *tile_x = g.tile_x;
    if (tile_y) *tile_y = g.tile_y;
    if (tile_rows) *tile_rows = g.rows_per_iter;
    if (blocks) *blocks = g.blocks;
    return LB_OK;
}

int lb_two_step_shape(const lb_params* p, int32_t* tile_x, int32_t* tile_y, int32_t* blocks)
{
    int rc = check_params(p);
    if (rc) return rc;
    const Geom g2 = make_geom2(*p, make_geom(*p));
    const bool on = use_two(*p, g2);
    if (tile_x) *tile_x = on ? g2.tile_x : 0;
    if (tile_y) *tile_y = on ? g2.tile_y : 0;
    if (blocks) *blocks = on ? g2.blocks : 0;
    return LB_OK;
}

int lb_tables(const lb_params* p, int8_t cx[24], int8_t cy[24], double K[24], double KE[25])
{
    if (!p) return fail(LB_ERR_INVALID, "params is NULL");
    if (!cx || !cy || !K || !KE) return fail(LB_ERR_INVALID, "NULL output table");
    for (int k = 0; k < 24; ++k) {
        cx[k] = (int8_t)kLX[k];
        cy[k] = (int8_t)kLY[k];
        K[k] = coupling(k, p->G1, p->G2);
        KE[1 + k] = K[k];
    }
    KE[0] = p->G1 * kW0 + p->G2 * kPS0;
    return LB_OK;
}

int lb_init(lb_ctx** out, const lb_params* p, void* workspace, size_t bytes,
            const double* rho_init, const double* ux_init, const double* uy_init,
            int inputs_on_device, void* hip_stream)
{
    if (!out) return fail(LB_ERR_INVALID, "out is NULL");
    *out = nullptr;
    int rc = check_params(p);
    if (rc) return rc;
    if (!workspace) return fail(LB_ERR_INVALID, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign)
        return fail(LB_ERR_INVALID, "workspace must be %zu-byte aligned", kAlign);
    if (!rho_init) return fail(LB_ERR_INVALID, "rho_init is NULL");
    const Geom g = make_geom(*p);
    const Layout L = make_layout(*p, g);
    if (bytes < L.total)
        return fail(LB_ERR_INVALID, "workspace too small: %zu < %zu bytes", bytes, L.total);
    const int64_t N = (int64_t)p->nx * p->ny;

    // Host inputs are validated right here; device inputs after a copy back.
    std::vector<double> host_rho;
    if (!inputs_on_device) {
        if ((rc = field_check_host(rho_init, N, true, "rho_init"))) return rc;
        if (ux_init && (rc = field_check_host(ux_init, N, false, "ux_init"))) return rc;
        if (uy_init && (rc = field_check_host(uy_init, N, false, "uy_init"))) return rc;
    }

    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev <= 0) return fail(LB_ERR_HIP, "no HIP device available");
    int dev = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return hip_fail(e, "hipGetDevice");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);

    if (inputs_on_device) {
        host_rho.resize(N);
        std::vector<double> hu;
        if ((e = hipMemcpyAsync(host_rho.data(), rho_init, N * sizeof(double), hipMemcpyDeviceToHost, st)))
            return hip_fail(e, "copy rho_init");
        if ((e = hipStreamSynchronize(st))) return hip_fail(e, "synchronise");
        if ((rc = field_check_host(host_rho.data(), N, true, "rho_init"))) return rc;
        for (const double* u : {ux_init, uy_init}) {
            if (!u) continue;
            hu.resize(N);
            if ((e = hipMemcpyAsync(hu.data(), u, N * sizeof(double), hipMemcpyDeviceToHost, st)))
                return hip_fail(e, "copy u_init");
            if ((e = hipStreamSynchronize(st))) return hip_fail(e, "synchronise");
            if ((rc = field_check_host(hu.data(), N, false, u == ux_init ? "ux_init" : "uy_init")))
                return rc;
        }
    }

    lb_ctx* c = new lb_ctx();
    c->p = *p;
    c->g = g;
    c->g2 = make_geom2(*p, g);
    c->two = use_two(*p, c->g2);
    c->coef = make_coef(*p);
    c->device = dev;
    c->stream = st;
    c->ws = static_cast<char*>(workspace);
    c->buf[0] = c->ws + L.buf[0];
    c->buf[1] = c->ws + L.buf[1];
    c->cur = 0;
    c->partials = reinterpret_cast<double*>(c->ws + L.partials);
    c->trace = reinterpret_cast<double*>(c->ws + L.trace);
    c->scalars = reinterpret_cast<double*>(c->ws + L.scalars);
    c->staging = reinterpret_cast<double*>(c->ws + L.staging);
    c->t = 0;
    c->trace_rows = 0;
    c->last_logged = -1;
    c->batch = nullptr;

    const double *r = rho_init, *u = ux_init, *v = uy_init;
    if (!inputs_on_device) {
        double* sr = c->staging;
        double* su = c->staging + N;
        double* sv = c->staging + 2 * N;
        e = hipMemcpyAsync(sr, rho_init, N * sizeof(double), hipMemcpyHostToDevice, st);
        if (!e && ux_init) e = hipMemcpyAsync(su, ux_init, N * sizeof(double), hipMemcpyHostToDevice, st);
        if (!e && uy_init) e = hipMemcpyAsync(sv, uy_init, N * sizeof(double), hipMemcpyHostToDevice, st);
        if (e) {
            delete c;
            return hip_fail(e, "copy initial fields");
        }
        r = sr;
        u = ux_init ? su : nullptr;
        v = uy_init ? sv : nullptr;
    }
    if ((e = lbk::launch_init(p->storage, r, u, v, c->buf[0], g, c->coef, st)) ||
        (e = hipStreamSynchronize(st))) {
        delete c;
        return hip_fail(e, "init kernel");
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_live.insert(c);
    }
    *out = c;
    return LB_OK;
}

int lb_step(lb_ctx* c, int64_t n)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (c->batch) return fail(LB_ERR_STATE, "this lattice belongs to a batch: step it with lb_batch_step");
    if (n < 0) return fail(LB_ERR_INVALID, "n must be >= 0");
    if (n == 0) return LB_OK;
    const int64_t le = c->p.log_every;
    // Rows this call appends: log points in [t, t+n) not recorded yet.  The
    // state at t+n itself is recorded by the step that leaves it (or by
    // lb_trace), so that logging always rides on a step.
    int64_t need = 0;
    if (le > 0) {
        const int64_t first = (c->t + le - 1) / le * le;
        if (first < c->t + n) need = (c->t + n - 1 - first) / le + 1;
        if (c->last_logged == c->t && c->t % le == 0) --need;
    }
    if (c->trace_rows + need > c->p.trace_cap)
        return fail(LB_ERR_STATE, "trace full: %lld rows recorded, %lld more needed, capacity %lld",
                    (long long)c->trace_rows, (long long)need, (long long)c->p.trace_cap);
    DeviceGuard dg(c->device);
    if (dg.err) return hip_fail(dg.err, "select device");

    for (int64_t s = 0; s < n; ++s) {
        const void* src = c->buf[c->cur];
        void* dst = c->buf[c->cur ^ 1];
        const bool log = le > 0 && c->t % le == 0 && c->last_logged != c->t;
        // Two plain steps in one launch when neither state is logged.
        if (c->two && !log && s + 1 < n && !(le > 0 && (c->t + 1) % le == 0)) {
            c->coef.step = (uint32_t)c->t;
            hipError_t e = lbk::launch_step2(c->p.storage, src, dst, c->g2, c->coef, c->stream);
            if (e) return hip_fail(e, "two-step kernel launch");
            c->cur ^= 1;
            c->t += 2;
            ++s;
            continue;
        }
        if (log) {
            // The logged step, then the reduction of its partials into the
            // trace row.  If only the reduction fails to launch, the step
            // itself was issued: the context follows it, without the row.
            c->coef.step = (uint32_t)c->t;
            hipError_t e = lbk::launch_step(c->p.storage, lbk::MODE_STEP_ENERGY, src, dst, c->g,
                                            c->coef, c->partials, c->stream);
            if (e) return hip_fail(e, "step kernel launch");
            c->cur ^= 1;
            ++c->t;
            e = lbk::launch_final(c->partials, c->g.blocks, (double)(c->t - 1),
                                  0.5 * (c->p.G1 + c->p.G2), c->trace + c->trace_rows * 6, c->stream);
            if (e) return hip_fail(e, "final reduction launch");
            c->last_logged = c->t - 1;
            ++c->trace_rows;
            continue;
        } else {
            c->coef.step = (uint32_t)c->t;
            hipError_t e = lbk::launch_step(c->p.storage, lbk::MODE_STEP, src, dst, c->g, c->coef,
                                            c->partials, c->stream);
            if (e) return hip_fail(e, "step kernel launch");
        }
        c->cur ^= 1;
        ++c->t;
    }
    return LB_OK;
}

int lb_time(lb_ctx* c, int64_t* t)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!t) return fail(LB_ERR_INVALID, "t is NULL");
    *t = c->t;
    return LB_OK;
}

int lb_moments(lb_ctx* c, double* rho, double* ux, double* uy, int on_device)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    DeviceGuard dg(c->device);
    if (dg.err) return hip_fail(dg.err, "select device");
    const int64_t N = (int64_t)c->p.nx * c->p.ny;
    hipError_t e;
    if (on_device) {
        if ((e = lbk::launch_moments(c->p.storage, c->buf[c->cur], c->g, c->coef, rho, ux, uy, c->stream)))
            return hip_fail(e, "moments kernel");
        return LB_OK;
    }
    double* s = c->staging;
    if ((e = lbk::launch_moments(c->p.storage, c->buf[c->cur], c->g, c->coef, rho ? s : nullptr,
                                 ux ? s + N : nullptr, uy ? s + 2 * N : nullptr, c->stream)))
        return hip_fail(e, "moments kernel");
    double* outs[3] = {rho, ux, uy};
    for (int q = 0; q < 3; ++q) {
        if (!outs[q]) continue;
        if ((e = hipMemcpyAsync(outs[q], s + q * N, N * sizeof(double), hipMemcpyDeviceToHost, c->stream)))
            return hip_fail(e, "copy moments");
    }
    if ((e = hipStreamSynchronize(c->stream))) return hip_fail(e, "synchronise");
    return LB_OK;
}

int lb_pseudo_energy(lb_ctx* c, double out[6])
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!out) return fail(LB_ERR_INVALID, "out is NULL");
    DeviceGuard dg(c->device);
    if (dg.err) return hip_fail(dg.err, "select device");
    if ((rc = energy_row(c, lbk::MODE_ENERGY, c->buf[c->cur], c->buf[c->cur ^ 1], c->scalars))) return rc;
    hipError_t e = hipMemcpyAsync(out, c->scalars, 6 * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (!e) e = hipStreamSynchronize(c->stream);
    if (e) return hip_fail(e, "copy energies");
    if (!rows_finite(out, 1)) return fail(LB_ERR_NONFINITE, "non-finite mass or energy at t = %lld", (long long)c->t);
    return LB_OK;
}

int lb_trace(lb_ctx* c, double* out, int64_t cap, int64_t* n_rows)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (cap < 0 || (cap > 0 && !out)) return fail(LB_ERR_INVALID, "bad output buffer");
    DeviceGuard dg(c->device);
    if (dg.err) return hip_fail(dg.err, "select device");
    // Record the current state first if it is a log point not yet recorded
    // and the trace has room.
    const int64_t le = c->p.log_every;
    if (!c->batch && le > 0 && c->t % le == 0 && c->last_logged != c->t &&
        c->trace_rows < c->p.trace_cap) {
        if ((rc = energy_row(c, lbk::MODE_ENERGY, c->buf[c->cur], c->buf[c->cur ^ 1],
                             c->trace + c->trace_rows * 6)))
            return rc;
        c->last_logged = c->t;
        ++c->trace_rows;
    }
    const int64_t rows = cap < c->trace_rows ? cap : c->trace_rows;
    hipError_t e = hipSuccess;
    if (rows > 0)
        e = hipMemcpyAsync(out, c->trace, rows * 6 * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (!e) e = hipStreamSynchronize(c->stream);
    if (e) return hip_fail(e, "copy trace");
    if (n_rows) *n_rows = c->trace_rows;
    if (!rows_finite(out, rows)) return fail(LB_ERR_NONFINITE, "non-finite value in the trace");
    return LB_OK;
}

int lb_get_state(lb_ctx* c, void* dst, int on_device)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!dst) return fail(LB_ERR_INVALID, "dst is NULL");
    DeviceGuard dg(c->device);
    if (dg.err) return hip_fail(dg.err, "select device");
    const size_t bytes = (size_t)9 * c->p.nx * c->p.ny * lbk::storage_bytes(c->p.storage);
    void* spare = c->buf[c->cur ^ 1];
    hipError_t e = lbk::launch_get_state(c->p.storage, c->buf[c->cur], on_device ? dst : spare, c->g, c->stream);
    if (e) return hip_fail(e, "state kernel");
    if (!on_device) {
        if ((e = hipMemcpyAsync(dst, spare, bytes, hipMemcpyDeviceToHost, c->stream)) ||
            (e = hipStreamSynchronize(c->stream)))
            return hip_fail(e, "copy state");
    }
    return LB_OK;
}

int lb_set_state(lb_ctx* c, const void* src, int on_device, int64_t t)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (c->batch) return fail(LB_ERR_STATE, "this lattice belongs to a batch");
    if (!src) return fail(LB_ERR_INVALID, "src is NULL");
    if (t < 0) return fail(LB_ERR_INVALID, "t must be >= 0");
    DeviceGuard dg(c->device);
    if (dg.err) return hip_fail(dg.err, "select device");
    const size_t bytes = (size_t)9 * c->p.nx * c->p.ny * lbk::storage_bytes(c->p.storage);
    void* spare = c->buf[c->cur ^ 1];
    hipError_t e = hipSuccess;
    const void* in = src;
    if (!on_device) {
        if ((e = hipMemcpyAsync(spare, src, bytes, hipMemcpyHostToDevice, c->stream)))
            return hip_fail(e, "copy state");
        in = spare;
    }
    // The permutation must not read and write one buffer: when the input was
    // staged in the spare buffer, write into the current one, else either.
    if ((e = lbk::launch_set_state(c->p.storage, in, c->buf[c->cur], c->g, c->stream)) ||
        (e = hipStreamSynchronize(c->stream)))
        return hip_fail(e, "state kernel");
    c->t = t;
    c->last_logged = -1;
    return LB_OK;
}

int lb_pseudo_energy_state(const lb_params* p, const void* state, double t, double out[6],
                           void* hip_stream)
{
    int rc = check_params(p);
    if (rc) return rc;
    if (!state) return fail(LB_ERR_INVALID, "state is NULL");
    if (!out) return fail(LB_ERR_INVALID, "out is NULL");
    if (!std::isfinite(t)) return fail(LB_ERR_INVALID, "t must be finite");
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev <= 0) return fail(LB_ERR_HIP, "no HIP device available");
    e = lbk::noalloc_energy(p->storage, state, p->nx, p->ny, make_coef(*p), t, 0.5 * (p->G1 + p->G2),
                            out, static_cast<hipStream_t>(hip_stream));
    if (e) return hip_fail(e, "energy of a population array");
    if (!rows_finite(out, 1)) return fail(LB_ERR_NONFINITE, "non-finite mass or energy");
    return LB_OK;
}

int lb_destroy(lb_ctx* c)
{
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!c || !g_live.count(c)) return fail(LB_ERR_STATE, "unknown or destroyed context");
        if (c->batch) return fail(LB_ERR_STATE, "this lattice belongs to a batch: use lb_batch_destroy");
        g_live.erase(c);
    }
    DeviceGuard dg(c->device);
    hipError_t e = hipStreamSynchronize(c->stream);
    delete c;
    if (e) return hip_fail(e, "synchronise");
    return LB_OK;
}

// ---------------------------------------------------------------------------
// Batches of independent lattices.
// ---------------------------------------------------------------------------
namespace {

std::set<lb_batch*> g_batches;

int check_batch(lb_batch* b)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (!b || !g_batches.count(b)) return fail(LB_ERR_STATE, "unknown or destroyed batch");
    return LB_OK;
}

// Workspace of a batch: descriptor table, tile -> lattice table, partials,
// then one single-lattice workspace per member.
struct BatchLayout {
    size_t desc, tile_lattice, tile_lattice2, partials;
    std::vector<size_t> member, member_bytes;
    size_t total;
    int tiles, tiles2, tiles2_cap, tile_y2;
    bool two;
    std::vector<Geom> geom2;
};

// Smallest two-step tile height of a batch: the two-step tile table is
// sized for it, so the height can change after initialisation.
constexpr int kBatchMinTile2 = 8;
constexpr int kBatchMaxTile2 = 64;

// Two-step geometry of a batch member: 128-lane tiles and a tile height
// shared by the batch.
Geom batch_geom2(const lb_params& p, int tile_y2)
{
    lb_params q = p;
    q.tile_x = 128;
    q.tile_y = std::min(tile_y2, p.ny);
    return make_geom2(q, make_geom(q));
}

int batch_layout(const lb_params* ps, int32_t count, BatchLayout* L)
{
    if (!ps) return fail(LB_ERR_INVALID, "params is NULL");
    if (count < 1 || count > 65536) return fail(LB_ERR_INVALID, "count must be in [1, 65536]");
    int rc;
    L->tiles = 0;
    Geom g0{};
    for (int32_t i = 0; i < count; ++i) {
        if ((rc = check_params(&ps[i]))) {
            return fail(rc, "lattice %d: %s", i, g_err.c_str());
        }
        const Geom g = make_geom(ps[i]);
        if (i == 0) g0 = g;
        if (ps[i].storage != ps[0].storage || g.tile_x != g0.tile_x ||
            g.rows_per_iter != g0.rows_per_iter || ps[i].log_every != ps[0].log_every ||
            ps[i].trace_cap != ps[0].trace_cap)
            return fail(LB_ERR_INVALID,
                        "lattice %d: storage, tile_x, tile_rows, log_every and trace_cap must "
                        "match lattice 0", i);
        if (ps[i].steps_per_launch != ps[0].steps_per_launch)
            return fail(LB_ERR_INVALID, "lattice %d: steps_per_launch must match lattice 0", i);
        if ((int64_t)L->tiles + g.blocks >= (int64_t(1) << 30))
            return fail(LB_ERR_INVALID, "too many tiles in the batch");
        L->tiles += g.blocks;
    }
    // Two steps per launch: FP32 or half storage, by default when the batch
    // as a whole fills tiles of >= 16 rows (the tallest of 48, 32, 24, 16
    // rows giving >= 1400 workgroups of 128 lanes; the lattices of a batch
    // are narrow, so the tiles stay 128 lanes wide).
    const int spl = ps[0].steps_per_launch;
    int tile_y2 = 0;
    for (int r : {48, 32, 24, 16}) {
        int64_t blocks = 0;
        for (int32_t i = 0; i < count; ++i) blocks += batch_geom2(ps[i], r).blocks;
        if (blocks >= 1400 && blocks < (int64_t(1) << 30)) {
            tile_y2 = r;
            break;
        }
    }
    const int st = ps[0].storage;
    L->two = (st == LB_F32 || st == LB_F16DEV) && (spl == 2 || (spl == 0 && tile_y2 >= 16));
    if (L->two && tile_y2 == 0) tile_y2 = 8;
    L->tile_y2 = L->two ? tile_y2 : 0;
    L->tiles2 = 0;
    L->tiles2_cap = 0;
    L->geom2.assign(count, Geom{});
    if (L->two)
        for (int32_t i = 0; i < count; ++i) {
            L->geom2[i] = batch_geom2(ps[i], tile_y2);
            L->tiles2 += L->geom2[i].blocks;
            L->tiles2_cap += batch_geom2(ps[i], kBatchMinTile2).blocks;
        }
    if ((int64_t)L->tiles2_cap >= (int64_t(1) << 30))
        return fail(LB_ERR_INVALID, "too many two-step tiles in the batch");
    size_t off = 0;
    L->desc = off;
    off += align_up(sizeof(lbk::BatchLattice) * count);
    L->tile_lattice = off;
    off += align_up(sizeof(int32_t) * L->tiles);
    L->tile_lattice2 = off;
    off += align_up(sizeof(int32_t) * L->tiles2_cap);
    L->partials = off;
    off += align_up(sizeof(double) * 4 * L->tiles);
    L->member.resize(count);
    L->member_bytes.resize(count);
    for (int32_t i = 0; i < count; ++i) {
        L->member[i] = off;
        L->member_bytes[i] = make_layout(ps[i], make_geom(ps[i])).total;
        off += L->member_bytes[i];
    }
    L->total = off;
    return LB_OK;
}

// One step of every lattice from buf[parity]; t is the step's time level
// (it seeds the half storage's stochastic rounding).
hipError_t batch_launch(lb_batch* b, int mode, int parity, int64_t t)
{
    return lbk::launch_step_batch(b->storage, mode, b->tile_x, b->rows_per_iter, b->min_tile_y, b->desc,
                                  b->tile_lattice, b->tiles, parity, (uint32_t)t, b->partials,
                                  b->stream);
}

// Buffer flips of a run of n plain steps: one per launch.
int batch_flips(const lb_batch* b, int64_t n)
{
    return (int)((b->two ? n / 2 + (n & 1) : n) & 1);
}

// n plain steps from buf[parity] at time t, launch by launch: pairs in the
// two-step kernel when the batch runs them so, then any odd step.  *done
// counts the steps whose launch was issued (all n unless one fails).
hipError_t batch_run(lb_batch* b, int64_t n, int parity, int64_t t, int64_t* done)
{
    int64_t j = 0;
    *done = 0;
    if (b->two)
        for (; j + 1 < n; j += 2, parity ^= 1) {
            hipError_t e = lbk::launch_step2_batch(b->storage, b->tile_x2, b->desc, b->tile_lattice2,
                                                   b->tiles2, parity, (uint32_t)(t + j), b->stream);
            if (e != hipSuccess) return e;
            *done = j + 2;
        }
    for (; j < n; ++j, parity ^= 1) {
        hipError_t e = batch_launch(b, lbk::MODE_STEP, parity, t + j);
        if (e != hipSuccess) return e;
        *done = j + 1;
    }
    return hipSuccess;
}

// n plain steps starting from the current parity, as one replay of a
// captured graph when the stream allows capture, else launch by launch.
// A graph keeps the time levels it was captured with, so batches whose
// rounding depends on them (half storage) never use graphs.  *done counts
// the steps issued.
hipError_t batch_plain(lb_batch* b, int64_t n, int64_t* done)
{
    *done = 0;
    if (b->use_graphs && n >= 2) {
        const auto key = std::make_pair(n, b->parity);
        auto it = b->graphs.find(key);
        if (it == b->graphs.end()) {
            hipGraph_t graph = nullptr;
            hipGraphExec_t exec = nullptr;
            hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                int64_t captured = 0;
                const hipError_t le = batch_run(b, n, b->parity, b->t, &captured);
                e = hipStreamEndCapture(b->stream, &graph);
                if (e == hipSuccess && le != hipSuccess) e = le;
            }
            if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            if (graph) (void)hipGraphDestroy(graph);
            if (e != hipSuccess) {
                // This stream cannot be captured: run launch by launch from now on.
                (void)hipGetLastError();
                b->use_graphs = false;
                return batch_plain(b, n, done);
            }
            it = b->graphs.emplace(key, exec).first;
        }
        const hipError_t e = hipGraphLaunch(it->second, b->stream);
        if (e == hipSuccess) *done = n;
        return e;
    }
    return batch_run(b, n, b->parity, b->t, done);
}

int batch_log(lb_batch* b, int mode)
{
    hipError_t e = batch_launch(b, mode, b->parity, b->t);
    if (!e)
        e = lbk::launch_final_batch(b->desc, (int)b->members.size(), b->partials, (double)b->t,
                                    b->trace_rows, b->stream);
    if (e) return hip_fail(e, "batched energy launch");
    b->last_logged = b->t;
    ++b->trace_rows;
    return LB_OK;
}

// n steps of the batch, logging where due; the batch's time level and
// parity follow every launch that was issued.
int batch_advance(lb_batch* b, int64_t n)
{
    const int64_t le = b->log_every;
    int rc;
    int64_t done = 0;
    while (done < n) {
        if (le > 0 && b->t % le == 0 && b->last_logged != b->t) {
            hipError_t e = batch_launch(b, lbk::MODE_STEP_ENERGY, b->parity, b->t);
            if (e) return hip_fail(e, "batched energy launch");
            b->parity ^= 1;
            ++b->t;
            ++done;
            e = lbk::launch_final_batch(b->desc, (int)b->members.size(), b->partials,
                                        (double)(b->t - 1), b->trace_rows, b->stream);
            if (e) return hip_fail(e, "batched energy reduction launch");
            b->last_logged = b->t - 1;
            ++b->trace_rows;
            continue;
        }
        int64_t run = n - done;
        if (le > 0) {
            const int64_t next = (b->t / le + 1) * le;
            if (next - b->t < run) run = next - b->t;
        }
        int64_t issued = 0;
        hipError_t e = batch_plain(b, run, &issued);
        // Launches issued: pairs first, then any odd step (as batch_run).
        b->parity ^= batch_flips(b, issued);
        b->t += issued;
        done += issued;
        if (e) return hip_fail(e, "batched step launch");
    }
    if (le > 0 && b->t % le == 0 && b->last_logged != b->t)
        if ((rc = batch_log(b, lbk::MODE_ENERGY))) return rc;
    return LB_OK;
}

void batch_sync_members(lb_batch* b)
{
    for (lb_ctx* c : b->members) {
        c->t = b->t;
        c->cur = b->parity;
        c->trace_rows = b->trace_rows;
        c->last_logged = b->last_logged;
    }
}

}  // namespace

size_t lb_batch_workspace_bytes(const lb_params* ps, int32_t count)
{
    BatchLayout L;
    if (batch_layout(ps, count, &L) != LB_OK) return 0;
    return L.total;
}

int lb_batch_init(lb_batch** out, const lb_params* ps, int32_t count, void* workspace,
                  size_t bytes, const double* const* rho_init, int inputs_on_device,
                  void* hip_stream)
{
    if (!out) return fail(LB_ERR_INVALID, "out is NULL");
    *out = nullptr;
    BatchLayout L;
    int rc = batch_layout(ps, count, &L);
    if (rc) return rc;
    if (!workspace) return fail(LB_ERR_INVALID, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign)
        return fail(LB_ERR_INVALID, "workspace must be %zu-byte aligned", kAlign);
    if (bytes < L.total) return fail(LB_ERR_INVALID, "workspace too small: %zu < %zu bytes", bytes, L.total);
    if (!rho_init) return fail(LB_ERR_INVALID, "rho_init is NULL");
    for (int32_t i = 0; i < count; ++i)
        if (!rho_init[i]) return fail(LB_ERR_INVALID, "rho_init[%d] is NULL", i);

    char* ws = static_cast<char*>(workspace);
    lb_batch* b = new lb_batch();
    b->stream = static_cast<hipStream_t>(hip_stream);
    std::vector<lbk::BatchLattice> desc(count);
    std::vector<int32_t> tl(L.tiles), tl2(L.tiles2);
    int tile = 0, tile2 = 0;
    for (int32_t i = 0; i < count; ++i) {
        lb_ctx* c = nullptr;
        rc = lb_init(&c, &ps[i], ws + L.member[i], L.member_bytes[i], rho_init[i], nullptr, nullptr,
                     inputs_on_device, hip_stream);
        if (rc) {
            std::string msg = g_err;
            for (lb_ctx* m : b->members) {
                m->batch = nullptr;
                lb_destroy(m);
            }
            delete b;
            return fail(rc, "lattice %d: %s", i, msg.c_str());
        }
        c->batch = b;
        b->members.push_back(c);
        lbk::BatchLattice& d = desc[i];
        std::memset(&d, 0, sizeof d);
        d.geom = c->g;
        d.coef = c->coef;
        lbk::coef_to_f32(c->coef, d.coef_f);
        d.buf[0] = c->buf[0];
        d.buf[1] = c->buf[1];
        d.trace = c->trace;
        d.half_A1 = 0.5 * (ps[i].G1 + ps[i].G2);
        d.tile_begin = tile;
        for (int j = 0; j < c->g.blocks; ++j) tl[tile + j] = i;
        tile += c->g.blocks;
        if (L.two) {
            d.geom2 = L.geom2[i];
            d.tile_begin2 = tile2;
            for (int j = 0; j < d.geom2.blocks; ++j) tl2[tile2 + j] = i;
            tile2 += d.geom2.blocks;
        }
    }
    lb_ctx* c0 = b->members[0];
    b->desc = reinterpret_cast<lbk::BatchLattice*>(ws + L.desc);
    b->tile_lattice = reinterpret_cast<int32_t*>(ws + L.tile_lattice);
    b->tile_lattice2 = reinterpret_cast<int32_t*>(ws + L.tile_lattice2);
    b->partials = reinterpret_cast<double*>(ws + L.partials);
    b->tiles = L.tiles;
    b->tiles2 = L.tiles2;
    b->two = L.two;
    b->tile_x2 = 128;
    b->tile_y2 = L.tile_y2;
    b->storage = ps[0].storage;
    b->tile_x = c0->g.tile_x;
    b->min_tile_y = c0->g.tile_y;
    for (lb_ctx* m : b->members) b->min_tile_y = std::min(b->min_tile_y, m->g.tile_y);
    b->rows_per_iter = c0->g.rows_per_iter;
    b->device = c0->device;
    b->parity = 0;
    b->t = 0;
    b->log_every = ps[0].log_every;
    b->trace_cap = ps[0].trace_cap;
    b->trace_rows = 0;
    b->last_logged = -1;
    b->use_graphs = b->stream != nullptr && b->storage != LB_F16DEV;
    b->params.assign(ps, ps + count);
    b->host_desc = desc;
    b->tiles2_cap = L.tiles2_cap;
    hipError_t e = hipMemcpyAsync(b->desc, desc.data(), sizeof(lbk::BatchLattice) * count,
                                  hipMemcpyHostToDevice, b->stream);
    if (!e) e = hipMemcpyAsync(b->tile_lattice, tl.data(), sizeof(int32_t) * L.tiles,
                               hipMemcpyHostToDevice, b->stream);
    if (!e && L.tiles2)
        e = hipMemcpyAsync(b->tile_lattice2, tl2.data(), sizeof(int32_t) * L.tiles2,
                           hipMemcpyHostToDevice, b->stream);
    if (!e) e = hipStreamSynchronize(b->stream);
    if (e) {
        for (lb_ctx* m : b->members) {
            m->batch = nullptr;
            lb_destroy(m);
        }
        delete b;
        return hip_fail(e, "copy batch tables");
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_batches.insert(b);
    }
    *out = b;
    return LB_OK;
}

int lb_batch_step(lb_batch* b, int64_t n)
{
    int rc = check_batch(b);
    if (rc) return rc;
    if (n < 0) return fail(LB_ERR_INVALID, "n must be >= 0");
    const int64_t le = b->log_every;
    // Rows this call appends: log points in [t, t+n] not recorded yet (the
    // state reached at t+n is recorded too).
    int64_t need = 0;
    if (le > 0) {
        const int64_t first = (b->t + le - 1) / le * le;
        if (first <= b->t + n) need = (b->t + n - first) / le + 1;
        if (b->last_logged == b->t && b->t % le == 0) --need;
    }
    if (b->trace_rows + need > b->trace_cap)
        return fail(LB_ERR_STATE, "trace full: %lld rows recorded, %lld more needed, capacity %lld",
                    (long long)b->trace_rows, (long long)need, (long long)b->trace_cap);
    DeviceGuard dg(b->device);
    if (dg.err) return hip_fail(dg.err, "select device");
    // On a launch failure the steps issued before it stand: the batch and
    // its member contexts are left at the time level they reached.
    rc = batch_advance(b, n);
    batch_sync_members(b);
    return rc;
}

int lb_batch_use_graphs(lb_batch* b, int enable)
{
    int rc = check_batch(b);
    if (rc) return rc;
    if (enable && !b->stream)
        return fail(LB_ERR_INVALID, "the null stream cannot be captured into a graph");
    if (enable && b->storage == LB_F16DEV)
        return fail(LB_ERR_INVALID, "half-storage batches seed their rounding with the time "
                                    "level and cannot replay captured graphs");
    b->use_graphs = enable != 0;
    return LB_OK;
}

int lb_batch_two_step_shape(lb_batch* b, int32_t* tile_x, int32_t* tile_y, int32_t* blocks)
{
    int rc = check_batch(b);
    if (rc) return rc;
    if (tile_x) *tile_x = b->two ? b->tile_x2 : 0;
    if (tile_y) *tile_y = b->two ? b->tile_y2 : 0;
    if (blocks) *blocks = b->two ? b->tiles2 : 0;
    return LB_OK;
}

int lb_batch_two_step_tile(lb_batch* b, int32_t tile_y)
{
    int rc = check_batch(b);
    if (rc) return rc;
    if (!b->two) return fail(LB_ERR_STATE, "this batch runs one step per launch");
    if (tile_y != 0 && (tile_y < kBatchMinTile2 || tile_y > kBatchMaxTile2))
        return fail(LB_ERR_INVALID, "tile_y must be 0 or in [%d, %d] (got %d)", kBatchMinTile2,
                    kBatchMaxTile2, tile_y);
    const int count = (int)b->members.size();
    BatchLayout L;
    if ((rc = batch_layout(b->params.data(), count, &L))) return rc;
    const int ty = tile_y ? tile_y : L.tile_y2;
    std::vector<lbk::BatchLattice> desc = b->host_desc;
    std::vector<int32_t> tl2;
    tl2.reserve(b->tiles2_cap);
    for (int i = 0; i < count; ++i) {
        desc[i].geom2 = batch_geom2(b->params[i], ty);
        desc[i].tile_begin2 = (int32_t)tl2.size();
        tl2.insert(tl2.end(), desc[i].geom2.blocks, i);
    }
    if ((int)tl2.size() > b->tiles2_cap) return fail(LB_ERR_INVALID, "two-step tile table too small");
    DeviceGuard dg(b->device);
    if (dg.err) return hip_fail(dg.err, "select device");
    // Work already issued reads the tables: let it finish before rewriting them.
    hipError_t e = hipStreamSynchronize(b->stream);
    if (!e) e = hipMemcpyAsync(b->desc, desc.data(), sizeof(lbk::BatchLattice) * count,
                               hipMemcpyHostToDevice, b->stream);
    if (!e) e = hipMemcpyAsync(b->tile_lattice2, tl2.data(), sizeof(int32_t) * tl2.size(),
                               hipMemcpyHostToDevice, b->stream);
    if (!e) e = hipStreamSynchronize(b->stream);
    if (e) return hip_fail(e, "copy batch tables");
    for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
    b->graphs.clear();  // captured launches carry the old grid
    b->host_desc = desc;
    b->tile_y2 = ty;
    b->tiles2 = (int)tl2.size();
    return LB_OK;
}

int lb_batch_member(lb_batch* b, int32_t i, lb_ctx** member)
{
    int rc = check_batch(b);
    if (rc) return rc;
    if (!member) return fail(LB_ERR_INVALID, "member is NULL");
    if (i < 0 || i >= (int32_t)b->members.size())
        return fail(LB_ERR_INVALID, "lattice index %d out of range", i);
    *member = b->members[i];
    return LB_OK;
}

int lb_batch_destroy(lb_batch* b)
{
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!b || !g_batches.count(b)) return fail(LB_ERR_STATE, "unknown or destroyed batch");
        g_batches.erase(b);
    }
    DeviceGuard dg(b->device);
    hipError_t e = hipStreamSynchronize(b->stream);
    for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
    for (lb_ctx* c : b->members) {
        std::lock_guard<std::mutex> lk(g_mu);
        g_live.erase(c);
        delete c;
    }
    delete b;
    if (e) return hip_fail(e, "synchronise");
    return LB_OK;
}


// ---------------------------------------------------------------------------
// Adjoint of a run: gradients of L = (E(T) - E*)^2 + beta A(T).
// ---------------------------------------------------------------------------
struct lb_adj {
    lb_ctx* fwd;          // the forward lattice (never handed out)
    lbk::AdjParams ap;
    int64_t T;
    int32_t every, nseg;
    size_t ckpt_bytes;    // one raw population buffer
    char* ckpt;           // nseg checkpoints, at t = 0, every, 2 every, ...
    char* tapes[2];       // two regions of `every` tape entries of 4 N values
    char* tapeT;          // tape entry of the state at T
    char* lam[2];         // 9 N values each
    char* g[2];           // N values each
    char* gF;             // 2 N values
    char* dir;            // 2 N values
    double* part;         // adj_blocks x 2: dL/dG from the steps
    double* partE;        // adj_blocks x 2: dE/dG at T
    double* partA;        // adj_blocks: interface measure
    double* red;          // 8 reduced values
    double* drho;         // N doubles
    int blocks;
    int32_t tape_of[2];   // segment whose tape each region holds, or -1
    bool have_forward;
    double E, A, E_target, beta, eps;
    // The backward pass re-steps segment s - 1 (taping it into region
    // (s - 1) & 1) on `side` while the adjoint steps of segment s run on
    // the context's stream; ev_r[b] marks region b taped, ev_a[b] region b
    // read.  Without a stream of its own (the null stream) both run in turn
    // on the context's stream.
    hipStream_t side;
    bool own_side;
    hipEvent_t ev_r[2], ev_a[2];
    // Full segments replay captured graphs: the taped re-step keyed by its
    // region, the adjoint steps by region and the parity of the adjoint
    // buffers at their start; valid for the couplings they were captured
    // with.
    std::map<int, hipGraphExec_t> tape_graphs, adj_graphs;
    double graph_G1, graph_G2;
    bool use_graphs;
};

namespace {

std::set<lb_adj*> g_adjs;

// n steps of the forward lattice on stream st, each also recording the tape
// entry of the state it leaves (entry j = state t + j) in `tape`.
hipError_t adj_tape_steps(lb_adj* a, int64_t n, char* tape, hipStream_t st)
{
    lb_ctx* c = a->fwd;
    const size_t entry = (size_t)4 * c->p.nx * c->p.ny * (a->ap.f64 ? 8 : 4);
    for (int64_t j = 0; j < n; ++j) {
        c->coef.step = (uint32_t)c->t;
        hipError_t e = lbk::launch_step(c->p.storage, lbk::MODE_STEP_TAPE, c->buf[c->cur],
                                        c->buf[c->cur ^ 1], c->g, c->coef,
                                        reinterpret_cast<double*>(tape + j * entry), st);
        if (e) return e;
        c->cur ^= 1;
        ++c->t;
    }
    return hipSuccess;
}

// n adjoint steps on stream st, from tape entry n - 1 down to 0, starting
// from adjoint buffer `cur`.
hipError_t adj_back_steps(lb_adj* a, int64_t n, const char* tape, int cur, hipStream_t st)
{
    const size_t entry = (size_t)4 * a->ap.nx * a->ap.ny * (a->ap.f64 ? 8 : 4);
    for (int64_t j = n - 1; j >= 0; --j) {
        hipError_t e = lbk::adj_step(a->ap, a->lam[cur], a->g[cur], tape + j * entry,
                                     a->lam[cur ^ 1], a->g[cur ^ 1], a->gF, a->part, st);
        if (e) return e;
        cur ^= 1;
    }
    return hipSuccess;
}

void adj_drop_graphs(lb_adj* a)
{
    for (auto& kv : a->tape_graphs) (void)hipGraphExecDestroy(kv.second);
    for (auto& kv : a->adj_graphs) (void)hipGraphExecDestroy(kv.second);
    a->tape_graphs.clear();
    a->adj_graphs.clear();
}

// Launch `work` on st, as one replay of a graph captured under `key` in
// `graphs` when graphs are in use (captured on first use), else directly.
hipError_t adj_replay(lb_adj* a, std::map<int, hipGraphExec_t>& graphs, int key, hipStream_t st,
                      const std::function<hipError_t()>& work)
{
    if (!a->use_graphs) return work();
    auto it = graphs.find(key);
    if (it == graphs.end()) {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            const hipError_t le = work();
            e = hipStreamEndCapture(st, &graph);
            if (e == hipSuccess && le != hipSuccess) e = le;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            // This stream cannot be captured: launch by launch from now on.
            (void)hipGetLastError();
            a->use_graphs = false;
            adj_drop_graphs(a);
            return work();
        }
        it = graphs.emplace(key, exec).first;
    }
    return hipGraphLaunch(it->second, st);
}

// Tape segment s into region s & 1 on the side stream (unless the region
// holds it already), once the adjoint steps that last read that region are
// done; marks the region taped.
hipError_t adj_restep(lb_adj* a, int32_t s)
{
    lb_ctx* c = a->fwd;
    const int b = s & 1;
    hipStream_t st = a->side;
    hipError_t e;
    if (a->tape_of[b] != s) {
        a->tape_of[b] = -1;
        const int64_t t0 = (int64_t)s * a->every;
        const int64_t n = a->T - t0 < a->every ? a->T - t0 : a->every;
        if ((e = hipStreamWaitEvent(st, a->ev_a[b], 0)) ||
            (e = hipMemcpyAsync(c->buf[0], a->ckpt + (size_t)s * align_up(a->ckpt_bytes), a->ckpt_bytes,
                                hipMemcpyDeviceToDevice, st)))
            return e;
        c->cur = 0;
        c->t = t0;
        auto work = [&] { return adj_tape_steps(a, n, a->tapes[b], st); };
        if (n == a->every) {
            e = adj_replay(a, a->tape_graphs, b, st, work);
            c->cur = (int)(n & 1);
            c->t = t0 + n;
        } else {
            e = work();
        }
        if (e) return e;
        a->tape_of[b] = s;
    }
    return hipEventRecord(a->ev_r[b], st);
}

// The adjoint steps of segment s on the context's stream, once its tape is
// in place; marks its region read.
hipError_t adj_backseg(lb_adj* a, int32_t s, int cur)
{
    const int b = s & 1;
    hipStream_t st = a->fwd->stream;
    const int64_t t0 = (int64_t)s * a->every;
    const int64_t n = a->T - t0 < a->every ? a->T - t0 : a->every;
    hipError_t e;
    if ((e = hipStreamWaitEvent(st, a->ev_r[b], 0))) return e;
    auto work = [&] { return adj_back_steps(a, n, a->tapes[b], cur, st); };
    e = n == a->every ? adj_replay(a, a->adj_graphs, b * 2 + cur, st, work) : work();
    if (e) return e;
    return hipEventRecord(a->ev_a[b], st);
}

int check_adj(lb_adj* a)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (!a || !g_adjs.count(a)) return fail(LB_ERR_STATE, "unknown or destroyed adjoint context");
    return LB_OK;
}

struct AdjLayout {
    lb_params fp;         // forward parameters: no trace
    size_t fwd, fwd_bytes, ckpt, ckpt_bytes, tape[2], tapeT, lam[2], g[2], gF, dir, part, partE, partA,
        red, drho, total;
    int32_t nseg;
    int blocks;
};

int adj_layout(const lb_params* p, int64_t nsteps, int32_t every, AdjLayout* L)
{
    int rc = check_params(p);
    if (rc) return rc;
    if (p->storage != LB_F64 && p->storage != LB_F32)
        return fail(LB_ERR_INVALID, "the adjoint needs LB_F64 or LB_F32 storage");
    if (nsteps < 0) return fail(LB_ERR_INVALID, "nsteps must be >= 0");
    if (every < 1) return fail(LB_ERR_INVALID, "checkpoint_every must be >= 1");
    // The adjoint kernels address their dense per-site arrays with 32-bit
    // byte offsets from a per-array base (8-byte values).
    if ((int64_t)p->nx * p->ny > (int64_t(1) << 29))
        return fail(LB_ERR_INVALID, "the adjoint supports at most 2^29 sites (got %lld)",
                    (long long)p->nx * p->ny);
    L->fp = *p;
    L->fp.log_every = 0;
    L->fp.trace_cap = 0;
    const Geom g = make_geom(L->fp);
    const Layout F = make_layout(L->fp, g);
    const int64_t N = (int64_t)p->nx * p->ny;
    const size_t es = p->storage == LB_F64 ? 8 : 4;
    const int64_t nseg = (nsteps + every - 1) / every;
    if (nseg > INT32_MAX) return fail(LB_ERR_INVALID, "too many checkpoints");
    L->nseg = (int32_t)nseg;
    L->blocks = lbk::adj_blocks(N);
    const int64_t seg_len = nsteps < every ? nsteps : every;
    size_t off = 0;
    L->fwd = off; L->fwd_bytes = F.total; off += align_up(F.total);
    L->ckpt_bytes = (size_t)9 * g.plane * es;
    L->ckpt = off; off += (size_t)nseg * align_up(L->ckpt_bytes);
    // Segment s is taped into region s & 1; a run of one segment keeps its
    // whole tape from the forward pass and needs only region 0.
    L->tape[0] = off; off += align_up((size_t)seg_len * 4 * N * es);
    L->tape[1] = L->tape[0];
    if (nseg > 1) { L->tape[1] = off; off += align_up((size_t)seg_len * 4 * N * es); }
    L->tapeT = off; off += align_up((size_t)4 * N * es);
    for (int q = 0; q < 2; ++q) { L->lam[q] = off; off += align_up((size_t)9 * N * es); }
    for (int q = 0; q < 2; ++q) { L->g[q] = off; off += align_up((size_t)N * es); }
    L->gF = off; off += align_up((size_t)2 * N * es);
    L->dir = off; off += align_up((size_t)2 * N * es);
    L->part = off; off += align_up((size_t)L->blocks * 2 * sizeof(double));
    L->partE = off; off += align_up((size_t)L->blocks * 2 * sizeof(double));
    L->partA = off; off += align_up((size_t)L->blocks * sizeof(double));
    L->red = off; off += align_up(8 * sizeof(double));
    L->drho = off; off += align_up((size_t)N * sizeof(double));
    L->total = off;
    return LB_OK;
}

}  // namespace

size_t lb_adj_workspace_bytes(const lb_params* p, int64_t nsteps, int32_t checkpoint_every)
{
    AdjLayout L;
    return adj_layout(p, nsteps, checkpoint_every, &L) ? 0 : L.total;
}

int lb_adj_init(lb_adj** out, const lb_params* p, int64_t nsteps, int32_t checkpoint_every,
                void* workspace, size_t bytes, void* hip_stream)
{
    if (!out) return fail(LB_ERR_INVALID, "out is NULL");
    *out = nullptr;
    AdjLayout L;
    int rc = adj_layout(p, nsteps, checkpoint_every, &L);
    if (rc) return rc;
    if (!workspace) return fail(LB_ERR_INVALID, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign)
        return fail(LB_ERR_INVALID, "workspace must be %zu-byte aligned", kAlign);
    if (bytes < L.total) return fail(LB_ERR_INVALID, "workspace too small: %zu < %zu bytes", bytes, L.total);
    char* ws = static_cast<char*>(workspace);
    const std::vector<double> ones((size_t)p->nx * p->ny, 1.0);
    lb_ctx* c = nullptr;
    if ((rc = lb_init(&c, &L.fp, ws + L.fwd, L.fwd_bytes, ones.data(), nullptr, nullptr, 0, hip_stream)))
        return rc;
    lb_adj* a = new lb_adj();
    a->fwd = c;
    a->ap.nx = p->nx;
    a->ap.ny = p->ny;
    a->ap.f64 = p->storage == LB_F64;
    a->ap.G1 = p->G1;
    a->ap.G2 = p->G2;
    a->ap.tau = p->tau;
    a->ap.sqrt_rho0 = std::sqrt(p->rho0);
    a->ap.inv_rho0 = 1.0 / p->rho0;
    a->T = nsteps;
    a->every = checkpoint_every;
    a->nseg = L.nseg;
    a->ckpt_bytes = L.ckpt_bytes;
    a->ckpt = ws + L.ckpt;
    for (int q = 0; q < 2; ++q) {
        a->tapes[q] = ws + L.tape[q];
        a->tape_of[q] = -1;
    }
    a->tapeT = ws + L.tapeT;
    for (int q = 0; q < 2; ++q) {
        a->lam[q] = ws + L.lam[q];
        a->g[q] = ws + L.g[q];
    }
    a->gF = ws + L.gF;
    a->dir = ws + L.dir;
    a->part = reinterpret_cast<double*>(ws + L.part);
    a->partE = reinterpret_cast<double*>(ws + L.partE);
    a->partA = reinterpret_cast<double*>(ws + L.partA);
    a->red = reinterpret_cast<double*>(ws + L.red);
    a->drho = reinterpret_cast<double*>(ws + L.drho);
    a->blocks = L.blocks;
    a->have_forward = false;
    a->graph_G1 = a->ap.G1;
    a->graph_G2 = a->ap.G2;
    a->use_graphs = hip_stream != nullptr;
    // The re-steps get a stream of their own (default priority) when the
    // context has one; on the null stream everything runs in turn.
    a->side = c->stream;
    a->own_side = false;
    a->ev_r[0] = a->ev_r[1] = a->ev_a[0] = a->ev_a[1] = nullptr;
    {
        DeviceGuard dg(c->device);
        hipError_t e = dg.err;
        for (hipEvent_t* ev : {&a->ev_r[0], &a->ev_r[1], &a->ev_a[0], &a->ev_a[1]})
            if (!e) e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
        if (!e && hip_stream) {
            e = hipStreamCreateWithFlags(&a->side, hipStreamNonBlocking);
            a->own_side = e == hipSuccess;
        }
        if (e) {
            for (hipEvent_t ev : {a->ev_r[0], a->ev_r[1], a->ev_a[0], a->ev_a[1]})
                if (ev) (void)hipEventDestroy(ev);
            delete a;
            lb_destroy(c);
            return hip_fail(e, "adjoint stream and events");
        }
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_adjs.insert(a);
    }
    *out = a;
    return LB_OK;
}

int lb_adj_forward(lb_adj* a, const double* rho_init, int on_device, double G1, double G2,
                   const lb_adj_loss* loss, double out[4])
{
    int rc = check_adj(a);
    if (rc) return rc;
    if (!rho_init || !loss || !out) return fail(LB_ERR_INVALID, "NULL argument");
    if (!std::isfinite(G1) || !std::isfinite(G2)) return fail(LB_ERR_INVALID, "G1, G2 must be finite");
    if (!std::isfinite(loss->E_target) || !std::isfinite(loss->beta) || !std::isfinite(loss->eps) ||
        !(loss->eps > 0.0))
        return fail(LB_ERR_INVALID, "loss: E_target and beta must be finite, eps finite and > 0");
    lb_ctx* c = a->fwd;
    DeviceGuard dg(c->device);
    if (dg.err) return hip_fail(dg.err, "select device");
    const int64_t N = (int64_t)c->p.nx * c->p.ny;
    hipStream_t st = c->stream;
    hipError_t e;
    // Validate the density on the host (device inputs are copied back).
    std::vector<double> host;
    const double* r = rho_init;
    if (on_device) {
        host.resize(N);
        if ((e = hipMemcpyAsync(host.data(), rho_init, N * sizeof(double), hipMemcpyDeviceToHost, st)) ||
            (e = hipStreamSynchronize(st)))
            return hip_fail(e, "copy rho_init");
        if ((rc = field_check_host(host.data(), N, true, "rho_init"))) return rc;
    } else {
        if ((rc = field_check_host(rho_init, N, true, "rho_init"))) return rc;
        if ((e = hipMemcpyAsync(c->staging, rho_init, N * sizeof(double), hipMemcpyHostToDevice, st)))
            return hip_fail(e, "copy rho_init");
        r = c->staging;
    }
    a->have_forward = false;
    a->tape_of[0] = a->tape_of[1] = -1;
    // Work left on the side stream by an earlier backward pass reads the
    // lattice buffers this run overwrites.
    if (a->own_side && (e = hipStreamSynchronize(a->side))) return hip_fail(e, "synchronise");
    c->p.G1 = G1;
    c->p.G2 = G2;
    c->coef = make_coef(c->p);
    a->ap.G1 = G1;
    a->ap.G2 = G2;
    c->cur = 0;
    c->t = 0;
    if ((e = lbk::launch_init(c->p.storage, r, nullptr, nullptr, c->buf[0], c->g, c->coef, st)))
        return hip_fail(e, "init kernel");
    for (int32_t s = 0; s < a->nseg; ++s) {
        if ((e = hipMemcpyAsync(a->ckpt + (size_t)s * align_up(a->ckpt_bytes), c->buf[c->cur],
                                a->ckpt_bytes, hipMemcpyDeviceToDevice, st)))
            return hip_fail(e, "checkpoint copy");
        const int64_t t0 = (int64_t)s * a->every;
        const int64_t n = a->T - t0 < a->every ? a->T - t0 : a->every;
        // The last segment is taped on the way, so the backward pass
        // starts without recomputing it.
        if (s + 1 < a->nseg) {
            if ((rc = lb_step(c, n))) return rc;
        } else {
            if ((e = adj_tape_steps(a, n, a->tapes[s & 1], st))) return hip_fail(e, "step kernel launch");
            a->tape_of[s & 1] = s;
        }
    }
    if ((e = lbk::adj_tape(c->p.storage, c->buf[c->cur], c->g, a->ap, a->tapeT, st)) ||
        (e = lbk::adj_area(a->ap, a->tapeT, loss->eps, a->dir, a->partA, st)) ||
        (e = lbk::adj_reduce(a->partA, a->blocks, 1, a->red, st)))
        return hip_fail(e, "interface measure");
    if ((rc = energy_row(c, lbk::MODE_ENERGY, c->buf[c->cur], c->buf[c->cur ^ 1], c->scalars))) return rc;
    double row[6], A = 0.0;
    if ((e = hipMemcpyAsync(row, c->scalars, sizeof row, hipMemcpyDeviceToHost, st)) ||
        (e = hipMemcpyAsync(&A, a->red, sizeof A, hipMemcpyDeviceToHost, st)) ||
        (e = hipStreamSynchronize(st)))
        return hip_fail(e, "copy loss terms");
    a->E = row[2] + row[3];
    a->A = A;
    a->E_target = loss->E_target;
    a->beta = loss->beta;
    a->eps = loss->eps;
    const double d = a->E - a->E_target;
    out[0] = d * d + a->beta * A;
    out[1] = a->E;
    out[2] = A;
    out[3] = row[1];
    if (!std::isfinite(out[0]) || !std::isfinite(out[3]))
        return fail(LB_ERR_NONFINITE, "non-finite loss or mass at T = %lld", (long long)a->T);
    a->have_forward = true;
    return LB_OK;
}

int lb_adj_backward(lb_adj* a, double dG[2], double* drho, int on_device)
{
    int rc = check_adj(a);
    if (rc) return rc;
    if (!dG || !drho) return fail(LB_ERR_INVALID, "NULL argument");
    if (!a->have_forward) return fail(LB_ERR_STATE, "lb_adj_backward needs a successful lb_adj_forward");
    lb_ctx* c = a->fwd;
    DeviceGuard dg(c->device);
    if (dg.err) return hip_fail(dg.err, "select device");
    const int64_t N = (int64_t)c->p.nx * c->p.ny;
    hipStream_t st = c->stream;
    const double two_dE = 2.0 * (a->E - a->E_target);
    hipError_t e;
    if ((e = lbk::adj_area(a->ap, a->tapeT, a->eps, a->dir, a->partA, st)) ||
        (e = lbk::adj_seed(a->ap, a->tapeT, a->dir, two_dE, a->beta, a->lam[0], a->g[0], a->partE, st)) ||
        (e = lbk::adj_zero(a->part, (int64_t)a->blocks * 2, st)))
        return hip_fail(e, "adjoint seed");
    if (a->use_graphs && (a->graph_G1 != a->ap.G1 || a->graph_G2 != a->ap.G2)) {
        adj_drop_graphs(a);
        a->graph_G1 = a->ap.G1;
        a->graph_G2 = a->ap.G2;
    }
    // Segments from the last to the first: the adjoint steps of segment s
    // (context stream) overlap the taped re-step of segment s - 1 (side
    // stream).  Both regions start out free, and the side stream starts
    // after the seed.
    if ((e = hipEventRecord(a->ev_a[0], st)) || (e = hipEventRecord(a->ev_a[1], st)))
        return hip_fail(e, "adjoint events");
    if (a->nseg > 0 && (e = adj_restep(a, a->nseg - 1))) return hip_fail(e, "adjoint re-step");
    int cur = 0;
    for (int32_t s = a->nseg - 1; s >= 0; --s) {
        if (s > 0 && (e = adj_restep(a, s - 1))) return hip_fail(e, "adjoint re-step");
        if ((e = adj_backseg(a, s, cur))) return hip_fail(e, "adjoint steps");
        const int64_t t0 = (int64_t)s * a->every;
        const int64_t n = a->T - t0 < a->every ? a->T - t0 : a->every;
        cur ^= (int)(n & 1);
    }
    double* dst = on_device ? drho : a->drho;
    if ((e = lbk::adj_rho_grad(a->ap, a->lam[cur], a->g[cur], dst, st)) ||
        (e = lbk::adj_reduce(a->part, a->blocks, 2, a->red + 2, st)) ||
        (e = lbk::adj_reduce(a->partE, a->blocks, 2, a->red + 4, st)))
        return hip_fail(e, "adjoint reductions");
    double r[4];
    if ((e = hipMemcpyAsync(r, a->red + 2, sizeof r, hipMemcpyDeviceToHost, st)))
        return hip_fail(e, "copy gradients");
    if (!on_device && (e = hipMemcpyAsync(drho, a->drho, N * sizeof(double), hipMemcpyDeviceToHost, st)))
        return hip_fail(e, "copy gradients");
    if ((e = hipStreamSynchronize(st))) return hip_fail(e, "synchronise");
    dG[0] = r[0] + two_dE * r[2];
    dG[1] = r[1] + two_dE * r[3];
    if (!std::isfinite(dG[0]) || !std::isfinite(dG[1]))
        return fail(LB_ERR_NONFINITE, "non-finite coupling gradient");
    return LB_OK;
}

int lb_adj_destroy(lb_adj* a)
{
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!a || !g_adjs.count(a)) return fail(LB_ERR_STATE, "unknown or destroyed adjoint context");
        g_adjs.erase(a);
    }
    if (a->own_side) (void)hipStreamSynchronize(a->side);
    const int rc = lb_destroy(a->fwd);  // synchronises the stream first
    adj_drop_graphs(a);
    if (a->own_side) (void)hipStreamDestroy(a->side);
    for (hipEvent_t ev : {a->ev_r[0], a->ev_r[1], a->ev_a[0], a->ev_a[1]}) (void)hipEventDestroy(ev);
    delete a;
    return rc;
}


// ---------------------------------------------------------------------------
// Structure factor of a density field.
// ---------------------------------------------------------------------------
struct lb_sk {
    lbk::SkPlan plan;
    std::vector<int64_t> counts;  // modes per shell
    double* rho;                  // device staging of host input, L*L doubles
    int device;
    hipStream_t stream;
};

namespace {

std::set<lb_sk*> g_sks;

int check_sk(lb_sk* s)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (!s || !g_sks.count(s)) return fail(LB_ERR_STATE, "unknown or destroyed structure-factor context");
    return LB_OK;
}

// Shell of a mode with l^2 + m^2 = q: the n with (2n-1)^2 <= 4q < (2n+1)^2
// (n - 1/2 <= sqrt(q) < n + 1/2), in integer arithmetic.
int64_t shell_of(int64_t q)
{
    int64_t n = (int64_t)std::floor(std::sqrt((double)q) + 0.5);
    while ((2 * n + 1) * (2 * n + 1) <= 4 * q) ++n;
    while (n > 0 && (2 * n - 1) * (2 * n - 1) > 4 * q) --n;
    return n;
}

int sk_check_L(int32_t L)
{
    if (L < 5 || L > lbk::kSkMaxL)
        return fail(LB_ERR_INVALID, "L must be in [5, %d] (got %d)", lbk::kSkMaxL, L);
    return LB_OK;
}

struct SkLayout {
    size_t tw, part, mean, z, zt, spec, idx, off, shell, kbar, rho, total;
    int32_t nshell, sum_blocks;
};

SkLayout sk_layout(int32_t L)
{
    SkLayout S;
    const int64_t N = (int64_t)L * L;
    const int64_t h = L / 2;  // largest |l| of an L-point transform
    S.nshell = (int32_t)shell_of(2 * h * h) + 1;
    S.sum_blocks = (int32_t)std::min<int64_t>(1024, (N + 255) / 256);
    size_t off = 0;
    S.tw = off; off += align_up((size_t)L * 2 * sizeof(double));
    S.part = off; off += align_up((size_t)S.sum_blocks * sizeof(double));
    S.mean = off; off += align_up(sizeof(double));
    S.z = off; off += align_up((size_t)N * 2 * sizeof(double));
    S.zt = off; off += align_up((size_t)N * 2 * sizeof(double));
    S.spec = off; off += align_up((size_t)N * sizeof(double));
    S.idx = off; off += align_up((size_t)N * sizeof(int32_t));
    S.off = off; off += align_up((size_t)(S.nshell + 1) * sizeof(int32_t));
    S.shell = off; off += align_up((size_t)S.nshell * sizeof(double));
    S.kbar = off; off += align_up(2 * sizeof(double));
    S.rho = off; off += align_up((size_t)N * sizeof(double));
    S.total = off;
    return S;
}

}  // namespace

int lb_sk_shells(int32_t L, int32_t* nshell)
{
    int rc = sk_check_L(L);
    if (rc) return rc;
    if (!nshell) return fail(LB_ERR_INVALID, "nshell is NULL");
    *nshell = sk_layout(L).nshell;
    return LB_OK;
}

size_t lb_sk_workspace_bytes(int32_t L)
{
    return sk_check_L(L) ? 0 : sk_layout(L).total;
}

int lb_sk_init(lb_sk** out, int32_t L, void* workspace, size_t bytes, void* hip_stream)
{
    if (!out) return fail(LB_ERR_INVALID, "out is NULL");
    *out = nullptr;
    int rc = sk_check_L(L);
    if (rc) return rc;
    const SkLayout S = sk_layout(L);
    if (!workspace) return fail(LB_ERR_INVALID, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign)
        return fail(LB_ERR_INVALID, "workspace must be %zu-byte aligned", kAlign);
    if (bytes < S.total) return fail(LB_ERR_INVALID, "workspace too small: %zu < %zu bytes", bytes, S.total);
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev <= 0) return fail(LB_ERR_HIP, "no HIP device available");
    int dev = 0;
    if ((e = hipGetDevice(&dev))) return hip_fail(e, "hipGetDevice");

    // Modes grouped by shell, each group in increasing index order (index
    // l * L + m of the [l][m] spectrum; l, m signed as in an FFT).
    const int64_t N = (int64_t)L * L;
    std::vector<int32_t> shell_n(N), off(S.nshell + 1, 0), idx(N);
    for (int32_t l = 0; l < L; ++l) {
        const int64_t ls = l <= (L - 1) / 2 ? l : l - L;
        for (int32_t m = 0; m < L; ++m) {
            const int64_t ms = m <= (L - 1) / 2 ? m : m - L;
            const int32_t n = (int32_t)shell_of(ls * ls + ms * ms);
            shell_n[(int64_t)l * L + m] = n;
            ++off[n + 1];
        }
    }
    for (int32_t n = 0; n < S.nshell; ++n) off[n + 1] += off[n];
    std::vector<int32_t> pos(off.begin(), off.end() - 1);
    for (int64_t i = 0; i < N; ++i) idx[pos[shell_n[i]]++] = (int32_t)i;

    char* ws = static_cast<char*>(workspace);
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    lb_sk* s = new lb_sk();
    lbk::SkPlan& p = s->plan;
    p.L = L;
    p.logL = 0;
    if ((L & (L - 1)) == 0)
        while ((1 << p.logL) < L) ++p.logL;
    p.nshell = S.nshell;
    p.sum_blocks = S.sum_blocks;
    p.tw = reinterpret_cast<double2*>(ws + S.tw);
    p.part = reinterpret_cast<double*>(ws + S.part);
    p.mean = reinterpret_cast<double*>(ws + S.mean);
    p.z = reinterpret_cast<double2*>(ws + S.z);
    p.zt = reinterpret_cast<double2*>(ws + S.zt);
    p.spec_t = reinterpret_cast<double*>(ws + S.spec);
    p.idx = reinterpret_cast<const int32_t*>(ws + S.idx);
    p.off = reinterpret_cast<const int32_t*>(ws + S.off);
    p.shell = reinterpret_cast<double*>(ws + S.shell);
    p.kbar = reinterpret_cast<double*>(ws + S.kbar);
    s->rho = reinterpret_cast<double*>(ws + S.rho);
    s->device = dev;
    s->stream = st;
    s->counts.resize(S.nshell);
    for (int32_t n = 0; n < S.nshell; ++n) s->counts[n] = off[n + 1] - off[n];
    if ((e = hipMemcpyAsync(ws + S.idx, idx.data(), N * sizeof(int32_t), hipMemcpyHostToDevice, st)) ||
        (e = hipMemcpyAsync(ws + S.off, off.data(), off.size() * sizeof(int32_t), hipMemcpyHostToDevice, st)) ||
        (e = lbk::sk_twiddles(p, st)) || (e = hipStreamSynchronize(st))) {
        delete s;
        return hip_fail(e, "copy shell tables");
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_sks.insert(s);
    }
    *out = s;
    return LB_OK;
}

int lb_sk_compute(lb_sk* s, const double* rho, int on_device, double* shell, int64_t* counts,
                  int32_t cap, double* kbar, double* spectrum)
{
    int rc = check_sk(s);
    if (rc) return rc;
    if (!rho) return fail(LB_ERR_INVALID, "rho is NULL");
    if (cap < 0 || (cap > 0 && !shell && !counts)) return fail(LB_ERR_INVALID, "bad shell outputs");
    const lbk::SkPlan& p = s->plan;
    const int64_t N = (int64_t)p.L * p.L;
    DeviceGuard dg(s->device);
    if (dg.err) return hip_fail(dg.err, "select device");
    hipError_t e;
    const double* r = rho;
    if (!on_device) {
        if ((rc = field_check_host(rho, N, false, "rho"))) return rc;
        if ((e = hipMemcpyAsync(s->rho, rho, N * sizeof(double), hipMemcpyHostToDevice, s->stream)))
            return hip_fail(e, "copy rho");
        r = s->rho;
    }
    if ((e = lbk::sk_compute(p, r, spectrum, s->stream))) return hip_fail(e, "structure-factor kernels");
    const int32_t n = cap < p.nshell ? cap : p.nshell;
    std::vector<double> sh(p.nshell);
    double kb[2] = {0.0, 0.0};
    if ((e = hipMemcpyAsync(sh.data(), p.shell, p.nshell * sizeof(double), hipMemcpyDeviceToHost, s->stream)) ||
        (e = hipMemcpyAsync(kb, p.kbar, sizeof kb, hipMemcpyDeviceToHost, s->stream)) ||
        (e = hipStreamSynchronize(s->stream)))
        return hip_fail(e, "copy shells");
    for (int32_t i = 0; i < n; ++i) {
        if (shell) shell[i] = sh[i];
        if (counts) counts[i] = s->counts[i];
    }
    if (kbar) *kbar = kb[0];
    for (double v : sh)
        if (!std::isfinite(v)) return fail(LB_ERR_NONFINITE, "non-finite structure factor");
    if (kbar && !std::isfinite(kb[0]))
        return fail(LB_ERR_NONFINITE, "kbar is not finite (uniform field: every S_n is 0)");
    return LB_OK;
}

int lb_sk_destroy(lb_sk* s)
{
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!s || !g_sks.count(s)) return fail(LB_ERR_STATE, "unknown or destroyed structure-factor context");
        g_sks.erase(s);
    }
    DeviceGuard dg(s->device);
    hipError_t e = hipStreamSynchronize(s->stream);
    delete s;
    if (e) return hip_fail(e, "synchronise");
    return LB_OK;
}

}  // extern "C"
