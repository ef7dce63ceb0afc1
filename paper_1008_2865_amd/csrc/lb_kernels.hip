// HIP kernels of the two-belt Shan-Chen lattice Boltzmann step for gfx950.
//
// The hot kernel, k_step, performs one full time step of eq. (1) of the
// paper for a strip of the lattice in a single pass over HBM:
//   pull-stream (read each population once from its upstream site),
//   moments, psi(rho), the 24-link two-belt force of eq. (FORCE),
//   BGK collision at the force-shifted velocity, and a coalesced store.
// The psi values the force needs (a 5x5 neighbourhood) are staged in a ring
// of six LDS rows: each workgroup owns `tile_x` columns (one per lane) and
// walks down `tile_y` rows; for every row it pulls the populations two rows
// ahead, turns them into psi for its columns plus a 2-column halo, and then
// evaluates force and collision for the row whose +-2 neighbourhood is
// complete.  The populations of the two rows in between stay in registers,
// so every population is read from HBM once per step except for the
// 2-row/2-column halo, whose re-reads hit L2.
//
// The same kernel optionally accumulates the section V observables
// (mass, E_s, E_m, sum psi^2) of the pre-collision state in double:
// per-lane sums, a 64-lane xor-shuffle tree, a fixed-order sum over the
// waves of the workgroup, one partial per workgroup, and a single-workgroup
// fixed-order final reduction (k_final).  No floating-point atomics are
// used, so results are bit-reproducible for a given launch shape.
#include "lb_internal.h"

#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>

namespace lbk {
namespace {

constexpr int kXcds = 8;  // gfx950: 8 XCDs, workgroups dispatched round-robin

// ---------------------------------------------------------------------------
// Storage policies: how a stored population becomes a value of the
// arithmetic type C and back.
// ---------------------------------------------------------------------------
struct PF64 {
    using S = double;
    using C = double;
    static constexpr bool kDev = false;
    __device__ static C ld(const S* p, C) { return *p; }
    __device__ static void st(S* p, C v, C) { *p = v; }
};
struct PF32 {
    using S = float;
    using C = float;
    static constexpr bool kDev = false;
    __device__ static C ld(const S* p, C) { return *p; }
    __device__ static void st(S* p, C v, C) { *p = v; }
};
// Half-precision deviation from the rest-state equilibrium w_i rho', rho'
// within 2^-20 of rho_ref (the offsets of dev_axis_offset).  Decoding is one
// rounding of off + h and encoding one rounding of v - off followed by the
// conversion (the step's collision forms the deviation itself, at tau = 1
// as one fma), in every kernel and at every call site, with contraction
// off, so that the same stored value decodes to the same float everywhere.
struct PF16 {
    using S = _Float16;
    using C = float;
    static constexpr bool kDev = true;
    __device__ static C ld(const S* p, C off)
    {
#pragma clang fp contract(off)
        return off + (C)(*p);
    }
    __device__ static void st(S* p, C v, C off)
    {
#pragma clang fp contract(off)
        C d = v - off;
        asm("" : "+v"(d));  // round d, then convert (never one fused rounding)
        *p = (S)d;
    }
};

// Counter-based hash of (site, step): 32 well-mixed bits (the murmur3
// finaliser applied to a combination of the coordinates).
__device__ __forceinline__ uint32_t site_hash(uint32_t x, uint32_t y, uint32_t t)
{
    uint32_t h = x * 0x9E3779B1u ^ (y + 0x7F4A7C15u) * 0x85EBCA77u ^ (t + 0x165667B1u) * 0xC2B2AE3Du;
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

template <typename C>
struct CoefT {
    C K1, K2, K4, K5, K8, KE0, tau, omega, sqrt_rho0, inv_rho0, rho_ref;
    C K4x2, K8x2;   // 2 K4 and 2 K8 (the |c_x| = 2 link pairs)
    uint32_t step;  // time step of the launch (seeds the stochastic rounding)
};

template <typename C>
__host__ __device__ CoefT<C> convert(const Coef& c)
{
    return CoefT<C>{(C)c.K1, (C)c.K2, (C)c.K4, (C)c.K5, (C)c.K8, (C)c.KE0,
                    (C)c.tau, (C)c.omega, (C)c.sqrt_rho0, (C)c.inv_rho0,
                    (C)c.rho_ref, (C)(2.0 * c.K4), (C)(2.0 * c.K8), c.step};
}

// Single-precision arithmetic uses the hardware exponential and reciprocal
// (about 1 ulp each; the single-precision path is held to the error the
// rounding of single precision itself produces, far above that).  Double
// precision uses the correctly rounded library functions.
__device__ __forceinline__ double exp_c(double v) { return exp(v); }
__device__ __forceinline__ float exp_c(float v) { return __expf(v); }
__device__ __forceinline__ double rcp_c(double v) { return 1.0 / v; }
__device__ __forceinline__ double fma_c(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_c(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ float rcp_c(float v) { return __builtin_amdgcn_rcpf(v); }

template <typename C>
__device__ __forceinline__ C psi_of(C rho, const CoefT<C>& k)
{
    return k.sqrt_rho0 * ((C)1 - exp_c(-rho * k.inv_rho0));
}

// Periodic wrap for v in [-n, 2n).
__device__ __forceinline__ int wrapi(int v, int n)
{
    v = v < 0 ? v + n : v;
    return v >= n ? v - n : v;
}

// Logical tile of hardware workgroup b: workgroups are dispatched to the
// XCDs round-robin, so give each XCD a contiguous run of logical tiles; the
// vertical neighbours of a tile, whose halo rows it re-reads, then share
// its L2.
__device__ __forceinline__ int xcd_remap(int b, int nb)
{
    const int per = nb / kXcds, rem = nb % kXcds;
    const int xcd = b % kXcds, idx = b / kXcds;
    return xcd < rem ? xcd * (per + 1) + idx
                     : rem * (per + 1) + (xcd - rem) * per + idx;
}

// Deviation offsets w_i rho' of the half storage (zero otherwise), and
// the decoding of a stored value.
template <class P>
struct Offs {
    using S = typename P::S;
    using C = typename P::C;
    C o0, o1, o2;  // rest, axis, diagonal
    C osum;        // o0 + 4 o1 + 4 o2, the offsets of all nine populations
    _Float16 one;  // 1, opaque to the compiler (see ld)
    __device__ Offs(C rho_ref)
    {
#pragma clang fp contract(off)
        // Offsets and their sum exact in single precision (dev_axis_offset).
        if constexpr (P::kDev) {
            static_assert(sizeof(C) == 4, "the half storage computes in single precision");
            o1 = dev_axis_offset(rho_ref);
            o0 = (C)4 * o1;
            o2 = (C)0.25 * o1;
            osum = (C)9 * o1;
        } else {
            o0 = o1 = o2 = osum = (C)0;
        }
        one = (_Float16)1;
        asm("" : "+v"(one));
    }
    __device__ C of(int i) const { return i == 0 ? o0 : (i < 5 ? o1 : o2); }
    // A stored value as the arithmetic type.  Half storage: off + h rounded
    // once, written as the fma h * 1 + off (the product is exact) with a
    // half-precision 1 the compiler cannot fold, so that it becomes a single
    // mixed-precision fma instead of a conversion and an add: the same value.
    __device__ C dec(S v, C off) const
    {
        if constexpr (P::kDev)
            return __builtin_fmaf((float)v, (float)one, off);
        else
            return v;
    }
    __device__ C ld(const S* p, C off) const { return dec(*p, off); }
};

// float -> half with stochastic rounding in hardware: the conversion adds
// random bits (the high bits of r) below the kept mantissa before
// truncating, so it rounds up with probability equal to the dropped
// fraction (unbiased), for normal and subnormal halves alike.
__device__ __forceinline__ _Float16 half_stochastic_hw(float v, uint32_t r)
{
    typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
    const half2_t z = {};
    return __builtin_amdgcn_cvt_sr_f16_f32(z, v, r, false)[0];
}

// Store the nine post-collision populations of one site.  For the half
// storage the moving populations are rounded to nearest, and the rest
// population absorbs their rounding errors (so the stored populations of a
// site sum to its density up to a single rounding) and is itself rounded
// stochastically: at a uniform state every site would otherwise make the
// same rounding error at every step and the total mass would drift.  For
// the half storage q[0] is the density and q[1..8] are already the
// deviations f*_i - w_i rho_ref (site_collide<..., true>).
template <class P>
__device__ __forceinline__ void store_site(typename P::S* const* pd, int at,
                                           const typename P::C q[9],
                                           const Offs<P>& o, uint32_t rnd)
{
    if constexpr (P::kDev) {
        // The rest population is stored as what the rounded moving
        // populations leave of rho, so the nine decoded values sum to rho up
        // to the rounding of the rest itself.
#pragma clang fp contract(off)
        float resid = q[0] - o.osum;
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            // Round the single-precision value, not the exact result of the
            // operation that formed it: the compiler may otherwise fuse that
            // fma with the conversion into one mixed-precision instruction
            // (a single rounding), in some kernels and not in others.
            float v = q[i];
            asm("" : "+v"(v));
            const _Float16 h = (_Float16)v;
            resid = __builtin_fmaf(-(float)h, (float)o.one, resid);  // exact product: resid - h
            pd[i][at] = h;
        }
        pd[0][at] = half_stochastic_hw(resid, rnd);
    } else {
#pragma unroll
        for (int i = 0; i < 9; ++i) P::st(pd[i] + at, q[i], o.of(i));
    }
}

// Pull the nine populations arriving at (x, y): f_i(x, t) = stored_i(x - c_i).
// xm/xp are the periodic columns x-1 / x+1.
template <class P>
__device__ __forceinline__ void pull(const typename P::S* const* pl,
                                     const Geom& g, int x, int xm, int xp,
                                     int y, const Offs<P>& o,
                                     typename P::C f[9])
{
    const int ym = y == 0 ? g.ny - 1 : y - 1;
    const int yp = y == g.ny - 1 ? 0 : y + 1;
    // Offsets inside one plane fit in 32 bits (the host checks it).
    const int r0 = y * g.pitch, rm = ym * g.pitch, rp = yp * g.pitch;
    f[0] = o.ld(pl[0] + r0 + x, o.o0);
    f[1] = o.ld(pl[1] + r0 + xm, o.o1);  // c = ( 1, 0)
    f[2] = o.ld(pl[2] + rm + x, o.o1);   // c = ( 0, 1)
    f[3] = o.ld(pl[3] + r0 + xp, o.o1);  // c = (-1, 0)
    f[4] = o.ld(pl[4] + rp + x, o.o1);   // c = ( 0,-1)
    f[5] = o.ld(pl[5] + rm + xm, o.o2);  // c = ( 1, 1)
    f[6] = o.ld(pl[6] + rm + xp, o.o2);  // c = (-1, 1)
    f[7] = o.ld(pl[7] + rp + xp, o.o2);  // c = (-1,-1)
    f[8] = o.ld(pl[8] + rp + xm, o.o2);  // c = ( 1,-1)
}

template <typename C>
__device__ __forceinline__ C density(const C f[9])
{
    return ((f[0] + (f[1] + f[3])) + (f[2] + f[4])) + ((f[5] + f[7]) + (f[6] + f[8]));
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// ---------------------------------------------------------------------------
// The fused step.  Threads = tile_x = NT; LDS ring of 6 psi rows of NT + 4.
// ---------------------------------------------------------------------------

// D2Q9 speed components, population order (0,0) (1,0) (0,1) (-1,0) (0,-1)
// (1,1) (-1,1) (-1,-1) (1,-1), packed two bits per population as c + 1 so a
// lane can look up its own population's speed without a memory table.
constexpr int kQCx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int kQCy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr unsigned pack_speeds(const int* c)
{
    unsigned v = 0;
    for (int i = 0; i < 9; ++i) v |= (unsigned)(c[i] + 1) << (2 * i);
    return v;
}
constexpr unsigned kCxPack = pack_speeds(kQCx);
constexpr unsigned kCyPack = pack_speeds(kQCy);
__device__ __forceinline__ int q_cx(int i) { return (int)((kCxPack >> (2 * i)) & 3u) - 1; }
__device__ __forceinline__ int q_cy(int i) { return (int)((kCyPack >> (2 * i)) & 3u) - 1; }
static_assert(((kCxPack >> 0) & 3u) == 1u && ((kCxPack >> 6) & 3u) == 0u &&
                  ((kCyPack >> 8) & 3u) == 0u && ((kCyPack >> 10) & 3u) == 2u,
              "speed packing");

// psi at the 25 sites of the force stencil around one site, read from five
// rows of a psi ring (rows y-2 .. y+2, LDS column c of the site), named by
// direction: e1 = psi(x+1, y), ne = psi(x+1, y+1), e2n = psi(x+2, y+1), ...
template <typename C>
struct Stencil {
    C p, e1, w1, n1, s1v, ne, nw, sw, se, e2, w2, n2, s2v, e2n, e2s, w2n, w2s, n2e, n2w, s2e, s2w,
        ne2, nw2, sw2, se2;
    __device__ __forceinline__ Stencil(const C* rm2, const C* rm1, const C* rc, const C* rp1,
                                       const C* rp2, int c)
        : p(rc[c]), e1(rc[c + 1]), w1(rc[c - 1]), n1(rp1[c]), s1v(rm1[c]), ne(rp1[c + 1]),
          nw(rp1[c - 1]), sw(rm1[c - 1]), se(rm1[c + 1]), e2(rc[c + 2]), w2(rc[c - 2]),
          n2(rp2[c]), s2v(rm2[c]), e2n(rp1[c + 2]), e2s(rm1[c + 2]), w2n(rp1[c - 2]),
          w2s(rm1[c - 2]), n2e(rp2[c + 1]), n2w(rp2[c - 1]), s2e(rm2[c + 1]), s2w(rm2[c - 1]),
          ne2(rp2[c + 2]), nw2(rp2[c - 2]), sw2(rm2[c - 2]), se2(rm2[c + 2])
    {
    }
};

// Force of eq. (FORCE) and the velocity-shift BGK collision at one site: R
// the pre-collision populations, st the psi stencil around the site, Q the
// post-collision populations; with kTape also the tape entry.  For the half
// storage (kDev) Q[0] is the density and Q[1..8] the deviations
// f*_i - w_i rho_ref from the offsets o1 (axis) and o2 (diagonal), which at
// tau = 1 come out of one fma each.  kOm = 1 or 0 states that tau is 1, or
// is not, for a caller that has branched on it already; -1 tests k.omega.
// Every kernel that updates a site calls this, so all of them round
// identically.
template <bool kTape, bool kDev, int kOm = -1, typename C>
__device__ __forceinline__ void site_collide(const C (&R)[9], const Stencil<C>& st, const CoefT<C>& k,
                                             C (&Q)[9], C* tp, C o1 = (C)0, C o2 = (C)0)
{
#pragma clang fp contract(off)
    // Multiply-adds are written out as fma and nothing else is contracted,
    // so every kernel variant (launch shape, batched or not, one or two
    // steps per launch, one or two sites per lane) rounds each site's update
    // identically.
    const C p = st.p;
    // eq. (FORCE): F = -psi(x) sum_k K_k psi(x + c_k) c_k, links paired with
    // their opposites.  The differences of opposite links off the axes
    // (|c|^2 = 2, 5, 8) enter both components, so they are formed once.
    const C d2a = st.ne - st.sw, d2b = st.se - st.nw;      // (1, 1), (1,-1)
    const C d8a = st.ne2 - st.sw2, d8b = st.se2 - st.nw2;  // (2, 2), (2,-2)
    const C d5a = st.e2n - st.w2s, d5b = st.e2s - st.w2n;  // (2, 1), (2,-1)
    const C d5c = st.n2e - st.s2w, d5d = st.n2w - st.s2e;  // (1, 2), (-1, 2)
    const C sumx =
        fma_c(k.K1, st.e1 - st.w1,
              fma_c(k.K2, d2a + d2b,
                    fma_c(k.K4x2, st.e2 - st.w2,
                          fma_c(k.K5, fma_c((C)2, d5a + d5b, d5c - d5d), k.K8x2 * (d8a + d8b)))));
    const C sumy =
        fma_c(k.K1, st.n1 - st.s1v,
              fma_c(k.K2, d2a - d2b,
                    fma_c(k.K4x2, st.n2 - st.s2v,
                          fma_c(k.K5, fma_c((C)2, d5c + d5d, d5a - d5b), k.K8x2 * (d8a - d8b)))));
    const C Fx = -p * sumx;
    const C Fy = -p * sumy;

    // BGK collision at u_eq = (j + tau F) / rho.
    const C rho = density(R);
    const C jx = (R[1] - R[3]) + ((R[5] - R[7]) + (R[8] - R[6]));
    const C jy = (R[2] - R[4]) + ((R[5] - R[7]) + (R[6] - R[8]));
    if (kTape) {
        tp[0] = rho;
        tp[1] = jx;
        tp[2] = jy;
        tp[3] = p;
    }
    const C inv = rcp_c(rho);
    const C ux = fma_c(k.tau, Fx, jx) * inv;
    const C uy = fma_c(k.tau, Fy, jy) * inv;
    // 1 - 1.5 u^2, and f_eq = w rho (1 - 1.5 u^2 + cu (3 + 4.5 cu)).
    const C base = fma_c((C)-1.5, fma_c(ux, ux, uy * uy), (C)1);
    const C r1 = rho * ((C)1 / (C)9);
    const C r2 = rho * ((C)1 / (C)36);
    auto poly = [&](C cu) { return fma_c(cu, fma_c((C)4.5, cu, (C)3), base); };
    const C pr[9] = {(C)0,        poly(ux),       poly(uy),        poly(-ux), poly(-uy),
                     poly(ux + uy), poly(uy - ux), poly(-ux - uy), poly(ux - uy)};
    auto wr = [&](int i) { return i < 5 ? r1 : r2; };
    auto off = [&](int i) { return i < 5 ? o1 : o2; };
    // f* = f + (f_eq - f) / tau; at tau = 1 (every run of the paper) that is
    // f_eq itself.  The branch is uniform.
    if (kOm == 0 || (kOm < 0 && k.omega != (C)1)) {
        const C om = k.omega;
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            Q[i] = fma_c(om, wr(i) * pr[i] - R[i], R[i]);
            if (kDev) Q[i] = Q[i] - off(i);
        }
    } else {
#pragma unroll
        for (int i = 1; i < 9; ++i) Q[i] = kDev ? fma_c(wr(i), pr[i], -off(i)) : wr(i) * pr[i];
    }
    // The collision conserves mass exactly; the rest population is taken
    // from that, so rounding cannot drift the mass.  The half storage forms
    // it when it rounds the moving populations: there Q[0] carries rho.
    if (kDev)
        Q[0] = rho;
    else
        Q[0] = rho - (((Q[1] + Q[3]) + (Q[2] + Q[4])) + ((Q[5] + Q[7]) + (Q[6] + Q[8])));
}

template <int J>
using Ic = std::integral_constant<int, J>;

// Lookahead of the row walk: the loads of a row are issued LEAD
// iterations before its psi is staged.  LEAD = 2 keeps two rows of loads in
// flight per wave (about 10 more registers in single precision, still 4
// waves per SIMD); its longer prologue only pays off on tall tiles.
constexpr int kLead2MinRows = 16;

// Plain steps of single-precision arithmetic with one row per stage have a
// LEAD = 2 variant.
template <class P, int RPI>
constexpr bool lead2_variant()
{
    return sizeof(typename P::C) == 4 && RPI == 1;
}

// One launch = one time step for a tile of NT columns (one lane each) by
// tile_y rows, walked RPI rows at a time.
template <class P, int NT, int MODE, int RPI, int LEAD>
__device__ __forceinline__ void
step_tile(const typename P::S* __restrict__ src, typename P::S* __restrict__ dst,
          const Geom& g, const CoefT<typename P::C>& k, double* __restrict__ partials,
          const int lb)
{
    using S = typename P::S;
    using C = typename P::C;
    constexpr bool kEnergy = MODE == MODE_STEP_ENERGY || MODE == MODE_ENERGY;
    constexpr bool kCollide = MODE != MODE_ENERGY;
    constexpr bool kTape = MODE == MODE_STEP_TAPE;
    constexpr int LW = NT + 4;
    constexpr int kWaves = NT / 64;
    constexpr int kHpw = 4 / kWaves;  // halo columns gathered per wave
    // psi ring: walk rows -2 .. RPI+1 around the rows being updated, plus
    // RPI rows being staged.  Population buffers: the RPI rows being
    // updated, the 2 rows after them (psi staged) and RPI lead rows whose
    // loads are in flight.
    constexpr int RS = 4 + 2 * RPI;
    constexpr int NB = 2 + RPI * (1 + LEAD);
    constexpr int U = NB / RPI;
    static_assert(NB % RPI == 0, "buffer rotation must be a whole number of iterations");
    static_assert(U <= 6, "the walk loop is unrolled at most 6 times");
    __shared__ C ring[RS][LW];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wid = tid >> 6;
    const int sx = lb % g.tiles_x;
    const int sy = lb / g.tiles_x;
    const int x0 = sx * NT;
    const int y0 = sy * g.tile_y;
    const int y1 = min(y0 + g.tile_y, g.ny);
    // Vertically adjacent tiles walk in opposite directions, so the rows
    // at a shared tile boundary are pulled by both tiles at about the same
    // time (both at the start or both at the end of their walk) and the
    // second pull of those halo rows is served by L2.
    const int dir = (sy & 1) ? -1 : 1;
    const int ystart = dir > 0 ? y0 : y1 - 1;
    const int nrows = y1 - y0;
    const int nx = g.nx, ny = g.ny;
    // Lattice row of walk row r (r may run up to 2 rows past either end).
    auto wrow = [&](int r) { return wrapi(ystart + r * dir, ny); };

    const S* pl[9];
    S* pd[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        pl[i] = src + (int64_t)i * g.plane;
        pd[i] = dst + (int64_t)i * g.plane;
    }
    const Offs<P> o(k.rho_ref);

    // This lane's column, LDS column tid + 2.
    const bool own = x0 + tid < nx;
    const int xc = (x0 + tid) % nx;
    const int xcm = xc == 0 ? nx - 1 : xc - 1;
    const int xcp = xc == nx - 1 ? 0 : xc + 1;

    // Halo: the 4 columns x0-2, x0-1, x0+NT, x0+NT+1 (LDS 0, 1, NT+2, NT+3).
    // Each wave gathers kHpw of them with a single load instruction per row:
    // lane j < 9 kHpw fetches population j % 9 of halo column j / 9 (the
    // other lanes repeat the last address), and the nine values are then
    // summed across lanes.  No lane-divergent loads.
    const int hj = lane < 9 * kHpw ? lane : 9 * kHpw - 1;
    const int hi = hj % 9;
    const int hcol = wid * kHpw + hj / 9;
    const int hlds = hcol < 2 ? hcol : NT + hcol;
    int hgx = (x0 - 2 + hlds - q_cx(hi)) % nx;
    hgx = hgx < 0 ? hgx + nx : hgx;
    const S* hp = src + (int64_t)hi * g.plane + hgx;
    const int hcy = q_cy(hi);
    const C hoff = o.of(hi);
    const int mcol = wid * kHpw + (lane < kHpw ? lane : 0);
    const int mlds = mcol < 2 ? mcol : NT + mcol;
    const int gbase = 9 * (lane < kHpw ? lane : 0);

    auto halo_load = [&](int y) -> C {
        // Row y - c_y of this lane's population, from the three row offsets
        // every lane of the wave shares.
        const int ym = y == 0 ? ny - 1 : y - 1;
        const int yp = y == ny - 1 ? 0 : y + 1;
        const int r = (hcy > 0 ? ym : (hcy < 0 ? yp : y)) * g.pitch;
        return o.ld(hp + r, hoff);
    };
    auto halo_psi = [&](C hv, int slot) {
        C h[9];
#pragma unroll
        for (int m = 0; m < 9; ++m) h[m] = __shfl(hv, gbase + m, 64);
        const C ps = psi_of(density(h), k);
        if (lane < kHpw) ring[slot][mlds] = ps;
    };

    // Walk row r lives in buffer r % NB (its halo value in Hh[r % NB]).
    // Each loop iteration advances RPI rows and the loop body is unrolled
    // U = NB / RPI times, so every
    // buffer index below is a compile-time constant: the rotation is a
    // renaming, never a register copy (a copy of a register whose load may
    // still be outstanding would force a wait on the memory counter, which
    // on this target also counts the stores just issued).
    C Bf[NB][9] = {};
    C Hh[NB] = {};

    // Prologue: psi of walk rows -2 .. RPI+1 into ring slots 0 .. RPI+3, the
    // populations of rows 0 .. RPI+1 into Bf[0 .. RPI+1], and the loads of
    // the first LEAD-1 stages of lead rows.  All rows are requested before
    // any is used, so the prologue costs one latency.
    {
        C T0[9], T1[9], hv[RPI + 4];
        pull<P>(pl, g, xc, xcm, xcp, wrow(-2), o, T0);
        pull<P>(pl, g, xc, xcm, xcp, wrow(-1), o, T1);
#pragma unroll
        for (int r = 0; r < RPI + 2; ++r) pull<P>(pl, g, xc, xcm, xcp, wrow(r), o, Bf[r]);
#pragma unroll
        for (int r = -2; r < RPI + 2; ++r) hv[r + 2] = halo_load(wrow(r));
#pragma unroll
        for (int r = RPI + 2; r < 2 + RPI * LEAD; ++r) {
            const int yl = r < nrows + 2 ? wrow(r) : wrow(0);
            pull<P>(pl, g, xc, xcm, xcp, yl, o, Bf[r % NB]);
            Hh[r % NB] = halo_load(yl);
        }
        ring[0][tid + 2] = psi_of(density(T0), k);
        ring[1][tid + 2] = psi_of(density(T1), k);
#pragma unroll
        for (int r = 0; r < RPI + 2; ++r) ring[r + 2][tid + 2] = psi_of(density(Bf[r]), k);
#pragma unroll
        for (int r = 0; r < RPI + 4; ++r) halo_psi(hv[r], r);
    }

    double aM = 0.0, aEs = 0.0, aEm = 0.0, aS2 = 0.0;

    // Software pipeline, per iteration (rows b .. b+RPI-1 along the walk):
    //   issue the loads of the rows LEAD stages ahead, b+2+RPI*LEAD .. |
    //   barrier | force + collision of rows b .. b+RPI-1 | psi of rows
    //   b+RPI+2 .. b+2RPI+1 (loaded LEAD-1 iterations ago) into the ring
    //   slots of rows b-RPI-2 .. b-3 | stores.
    // The loads overlap LEAD barriers and rounds of arithmetic; the stores
    // overlap the next iteration's barrier and arithmetic.  The overwritten
    // slots were last read in the previous iteration, before this barrier.
    // Lead rows past the end of the walk re-read row b instead (an L2 hit),
    // so no load is conditional.
    auto group = [&](auto Jc, int it, int s0) {
        constexpr int J = decltype(Jc)::value;
        const int b = it * RPI;
#pragma unroll
        for (int m = 0; m < RPI; ++m) {
            const int r = b + 2 + RPI * LEAD + m;
            const int yl = r < nrows + 2 ? wrow(r) : wrow(b);
            pull<P>(pl, g, xc, xcm, xcp, yl, o, Bf[(J * RPI + 2 + RPI * LEAD + m) % NB]);
            Hh[(J * RPI + 2 + RPI * LEAD + m) % NB] = halo_load(yl);
        }
        __syncthreads();

        C q[RPI][9];
        C tp[RPI][4];  // tape entry (MODE_STEP_TAPE)
        C anchor = (C)0;
#pragma unroll
        for (int m = 0; m < RPI; ++m) {
            const C(&R)[9] = Bf[(J * RPI + m) % NB];
            if (m > 0 && b + m >= nrows) break;
            // Ring rows y-2 .. y+2 of lattice row y = walk row b+m.
            auto slot = [&](int dy) {
                int v = s0 + m + 2 + dy * dir;
                return v >= RS ? v - RS : v;
            };
            const C* rm2 = ring[slot(-2)];
            const C* rm1 = ring[slot(-1)];
            const C* rc = ring[slot(0)];
            const C* rp1 = ring[slot(1)];
            const C* rp2 = ring[slot(2)];
            const int c = tid + 2;

            const Stencil<C> st(rm2, rm1, rc, rp1, rp2, c);
            const C p = st.p;

            if (kEnergy && own) {
                // No contraction here: the energies must round identically
                // in every kernel variant that computes them (the step
                // that also logs, the energy-only pass, the batched kernel).
#pragma clang fp contract(off)
                const C S1 = (st.e1 + st.w1) + (st.n1 + st.s1v);
                const C S2 = (st.ne + st.sw) + (st.nw + st.se);
                const C S4 = (st.e2 + st.w2) + (st.n2 + st.s2v);
                const C S5 = ((st.e2n + st.w2s) + (st.e2s + st.w2n)) + ((st.n2e + st.s2w) + (st.n2w + st.s2e));
                const C S8 = (st.ne2 + st.sw2) + (st.nw2 + st.se2);
                const C es = (C)0.5 * p * (k.KE0 * p + k.K1 * S1 + k.K2 * S2);
                const C em = (C)0.5 * p * (k.K4 * S4 + k.K5 * S5 + k.K8 * S8);
                aM += (double)density(R);
                aEs += (double)es;
                aEm += (double)em;
                aS2 += (double)p * (double)p;
            }

            if (kCollide) {
                site_collide<kTape, P::kDev>(R, st, k, q[m], tp[m], o.o1, o.o2);
                if (m == 0) anchor = q[m][1];
            } else if (m == 0) {
                anchor = p;
            }
        }

        // Stage psi of the lead rows (their loads have had the barrier and
        // the arithmetic above to arrive).  Rows past the end of the walk
        // write slots nobody reads any more.  The empty asm statements tie
        // the lead-row registers to the result of the arithmetic, so the
        // compiler cannot hoist this staging (and the wait for those loads)
        // above the arithmetic; the fence after it keeps the stores below,
        // so the wait does not also cover this iteration's stores.
#pragma unroll
        for (int m = 0; m < RPI; ++m) {
            C(&NF)[9] = Bf[(J * RPI + RPI + 2 + m) % NB];
            C& HF = Hh[(J * RPI + RPI + 2 + m) % NB];
#pragma unroll
            for (int i = 0; i < 9; ++i) asm volatile("" : "+v"(NF[i]) : "v"(anchor));
            asm volatile("" : "+v"(HF) : "v"(anchor));
            int sl = s0 + RPI + 4 + m;
            sl = sl >= RS ? sl - RS : sl;
            ring[sl][tid + 2] = psi_of(density(NF), k);
            halo_psi(HF, sl);
        }
        __builtin_amdgcn_sched_barrier(0);

        if (kCollide && own) {
#pragma unroll
            for (int m = 0; m < RPI; ++m) {
                if (m > 0 && b + m >= nrows) break;
                const int yw = wrow(b + m);
                const uint32_t rnd = P::kDev ? site_hash(xc, yw, k.step) : 0u;
                store_site<P>(pd, yw * g.pitch + xc, q[m], o, rnd);
                if (kTape) {
                    C* tape = reinterpret_cast<C*>(partials);
                    const int64_t N = (int64_t)nx * ny, si = (int64_t)yw * nx + xc;
#pragma unroll
                    for (int v = 0; v < 4; ++v) tape[v * N + si] = tp[m][v];
                }
            }
        }
    };

    auto step_slot = [](int s) { return s + RPI >= RS ? s + RPI - RS : s + RPI; };
    int s0 = 0;  // ring slot of walk row b - 2
#pragma unroll 1
    for (int it = 0;;) {
        group(Ic<0>{}, it, s0);
        s0 = step_slot(s0);
        if (++it * RPI >= nrows) break;
        group(Ic<1 % U>{}, it, s0);
        s0 = step_slot(s0);
        if (++it * RPI >= nrows) break;
        group(Ic<2 % U>{}, it, s0);
        s0 = step_slot(s0);
        if (++it * RPI >= nrows) break;
        if constexpr (U >= 4) {
            group(Ic<3 % U>{}, it, s0);
            s0 = step_slot(s0);
            if (++it * RPI >= nrows) break;
        }
        if constexpr (U >= 5) {
            group(Ic<4 % U>{}, it, s0);
            s0 = step_slot(s0);
            if (++it * RPI >= nrows) break;
        }
        if constexpr (U >= 6) {
            group(Ic<5 % U>{}, it, s0);
            s0 = step_slot(s0);
            if (++it * RPI >= nrows) break;
        }
    }

    if (kEnergy) {
        __shared__ double red[4][kWaves];
        double v[4] = {aM, aEs, aEm, aS2};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            v[q] = wave_sum(v[q]);
            if (lane == 0) red[q][wid] = v[q];
        }
        __syncthreads();
        if (tid < 4) {
            double s = 0.0;
            for (int w = 0; w < kWaves; ++w) s += red[tid][w];
            partials[(int64_t)lb * 4 + tid] = s;
        }
    }
}

// ---------------------------------------------------------------------------
// Two time steps per launch (temporal blocking) for plain steps of the
// single-precision and half storages.  A tile of NT lanes produces NT - 6 output columns x0 .. x0+W-1 of
// step t+2 for tile_y rows.  Level 1 is the one-step row walk above on the
// NT columns x0-3 .. x0+NT-4 and on rows -3 .. nrows+2 of the tile (walk
// order); its post-collision rows go to a 4-row LDS ring instead of memory.
// Level 2 trails it: at walk row p it pulls the pre-collision populations of
// row p-2 at t+1 from that ring (rows p-3 .. p-1, lanes l-1 .. l+1), stages
// their psi, and, after the row's barrier, applies the same force and
// collision (site_collide, so every site rounds as in two one-step
// launches) to row p-4, which it stores.  One barrier per walk row: every
// LDS row an iteration reads was written before the previous barrier, and
// the slots written between two barriers are not read between them (the
// rings are deep enough).  Global traffic per two steps is one read and one
// write of the populations, plus halo rows and columns that neighbouring
// tiles also read.
// ---------------------------------------------------------------------------
// LDS of a two-step workgroup, declared once per kernel so that the walks
// for tau = 1 and for other tau share it.
template <class P, int NT>
struct Step2Smem {
    static constexpr int RS = 6, RS2 = 6, NF = 4;
    typename P::C ring[RS][NT + 4];   // psi at t, level-1 rows p-2 .. p+3
    typename P::C ring2[RS2][NT + 4]; // psi at t+1, rows p-7 .. p-2
    // Post-collision populations of step t+1, in the storage type and
    // rounded exactly as a one-step launch stores them.
    typename P::S fs[NF][9][NT];
};

// Issue priority of a wave for one walk row.  Among waves of equal
// priority the arbiter picks the oldest, so the workgroups a CU receives
// first run ahead of the ones it receives last, which then finish alone
// (timed per workgroup at 2048^2: 61 us for the first resident slot, 74 us
// for the last, against an 82 us launch).  Drawing each row's priority from
// a hash of the row and the workgroup keeps any wave from holding the lead:
// launches 0.4% (2048^2) to 1.7% (half storage 8192^2) shorter.  The
// priority orders issue only; results are unaffected.
__device__ __forceinline__ void set_row_priority(int it)
{
    const uint32_t h = ((uint32_t)it * 0x9E3779B1u + blockIdx.x * 0x85EBCA77u) >> 30;
    switch (h) {
    case 0: __builtin_amdgcn_s_setprio(0); break;
    case 1: __builtin_amdgcn_s_setprio(1); break;
    case 2: __builtin_amdgcn_s_setprio(2); break;
    default: __builtin_amdgcn_s_setprio(3); break;
    }
}

template <class P, int NT, int kOm>
__device__ __forceinline__ void
step2_tile(const typename P::S* __restrict__ src, typename P::S* __restrict__ dst,
           const Geom& g, const CoefT<typename P::C>& k, const int lb, Step2Smem<P, NT>& sm)
{
    using S = typename P::S;
    using C = typename P::C;
    constexpr int W = NT - 6;           // output columns of the tile
    constexpr int LW = NT + 4;          // psi rings: lanes plus 2 columns each side
    constexpr int kWaves = NT / 64;
    constexpr int kHpw = 4 / kWaves;
    constexpr int RS = Step2Smem<P, NT>::RS, RS2 = Step2Smem<P, NT>::RS2, NF = Step2Smem<P, NT>::NF;
    C (&ring)[RS][LW] = sm.ring;
    C (&ring2)[RS2][LW] = sm.ring2;
    S (&fs)[NF][9][NT] = sm.fs;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wid = tid >> 6;
    const int sx = lb % g.tiles_x;
    const int sy = lb / g.tiles_x;
    const int x0 = sx * W;              // first output column
    const int y0 = sy * g.tile_y;
    const int y1 = min(y0 + g.tile_y, g.ny);
    const int dir = (sy & 1) ? -1 : 1;
    const int ystart = dir > 0 ? y0 : y1 - 1;
    const int nrows = y1 - y0;
    const int nx = g.nx, ny = g.ny;
    auto modn = [](int v, int n) { v %= n; return v < 0 ? v + n : v; };
    // Lattice row of walk row r.  r runs from -5 to nrows + 4, so
    // ystart + r dir lies in [y0 - 5, y1 + 4], within [-ny, 2 ny) for
    // ny >= 5: one conditional add or subtract wraps it (a modulo by a
    // value unknown at compile time costs a long scalar sequence per row).
    auto wrow = [&](int r) { return wrapi(ystart + r * dir, ny); };

    const S* pl[9];
    S* pd[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        pl[i] = src + (int64_t)i * g.plane;
        pd[i] = dst + (int64_t)i * g.plane;
    }
    const Offs<P> o(k.rho_ref);
    CoefT<C> k2 = k;
    k2.step = k.step + 1;

    // Level-1 column of this lane (LDS column tid + 2): x0 - 3 + tid.
    const int xb = x0 - 3;
    const int xc = modn(xb + tid, nx);
    const int xcm = xc == 0 ? nx - 1 : xc - 1;
    const int xcp = xc == nx - 1 ? 0 : xc + 1;
    // Level-2 output: lanes 3 .. 3+W-1, column x0 + tid - 3.
    const bool own2 = tid >= 3 && tid < 3 + W && x0 + tid - 3 < nx;

    // Halo columns of level 1 (xb-2, xb-1, xb+NT, xb+NT+1), gathered as in
    // the one-step walk.
    const int hj = lane < 9 * kHpw ? lane : 9 * kHpw - 1;
    const int hi = hj % 9;
    const int hcol = wid * kHpw + hj / 9;
    const int hlds = hcol < 2 ? hcol : NT + hcol;
    const int hgx = modn(xb - 2 + hlds - q_cx(hi), nx);
    const S* hp = src + (int64_t)hi * g.plane + hgx;
    const int hcy = q_cy(hi);
    const C hoff = o.of(hi);
    const int mcol = wid * kHpw + (lane < kHpw ? lane : 0);
    const int mlds = mcol < 2 ? mcol : NT + mcol;
    const int gbase = 9 * (lane < kHpw ? lane : 0);
    auto halo_load = [&](int y) -> C {
        const int ym = y == 0 ? ny - 1 : y - 1;
        const int yp = y == ny - 1 ? 0 : y + 1;
        const int r = (hcy > 0 ? ym : (hcy < 0 ? yp : y)) * g.pitch;
        return o.ld(hp + r, hoff);
    };
    auto halo_psi = [&](C hv, int slot) {
        C h[9];
#pragma unroll
        for (int m = 0; m < 9; ++m) h[m] = __shfl(hv, gbase + m, 64);
        const C ps = psi_of(density(h), k);
        if (lane < kHpw) ring[slot][mlds] = ps;
    };

    // Level-1 walk row p lives in Bf[(p + 3) % NBF] (p >= -3); the level-2
    // pre-collision row formed at iteration it in F2[(it + 2) % NBF].  The
    // loads of a row are written LEAD iterations before its psi is staged:
    // one for single precision; two for the half storage, whose loop then
    // unrolls five-fold.  The compiler moves those loads back next to their
    // use (the source is read-only), and for the five-fold loop it needs
    // fewer registers (165 against 173: three waves per SIMD, not two).
    constexpr int LEAD = P::kDev ? 2 : 1;
    constexpr int NBF = 3 + LEAD;
    C Bf[NBF][9] = {};
    C Hh[NBF] = {};
    C F2[NBF][9] = {};

    // Prologue: psi at t of walk rows -5 .. -1 into ring slots 0 .. 4 and
    // the populations of rows -3 .. -1 into Bf[0 .. 2].
    {
        C T0[9], T1[9], hv[5];
        pull<P>(pl, g, xc, xcm, xcp, wrow(-5), o, T0);
        pull<P>(pl, g, xc, xcm, xcp, wrow(-4), o, T1);
#pragma unroll
        for (int r = 0; r < 3; ++r) pull<P>(pl, g, xc, xcm, xcp, wrow(r - 3), o, Bf[r]);
#pragma unroll
        for (int r = 0; r < 5; ++r) hv[r] = halo_load(wrow(r - 5));
        ring[0][tid + 2] = psi_of(density(T0), k);
        ring[1][tid + 2] = psi_of(density(T1), k);
#pragma unroll
        for (int r = 0; r < 3; ++r) ring[r + 2][tid + 2] = psi_of(density(Bf[r]), k);
#pragma unroll
        for (int r = 0; r < 5; ++r) halo_psi(hv[r], r);
        // Rows 0 .. LEAD - 2: their loads stay in flight into the walk.
#pragma unroll
        for (int r = 0; r < LEAD - 1; ++r) {
            pull<P>(pl, g, xc, xcm, xcp, wrow(r), o, Bf[3 + r]);
            Hh[3 + r] = halo_load(wrow(r));
        }
    }
    __syncthreads();

    // One iteration per level-1 row p = it - 3, it = 0 .. nrows + 6.
    auto group = [&](auto Jc, int it, int s0) {
        constexpr int J = decltype(Jc)::value;  // it % NBF
        const int p = it - 3;
        set_row_priority(it);
        // ring2 holds walk row r in slot (r + 12) % RS2.  s0 = it % RS,
        // so walk row p - 6 + k sits in slot b2 + k (mod RS2), k = 0 .. 4,
        // with no division.
        const int b2 = s0 >= 3 ? s0 - 3 : s0 + 3;
        auto slot2 = [&](int kk) {
            const int v = b2 + kk;
            return v >= RS2 ? v - RS2 : v;
        };
        // Lead row p + 2 + LEAD (psi at t is needed up to row nrows + 4).
        {
            const int r = p + 2 + LEAD;
            const int yl = r < nrows + 5 ? wrow(r) : wrow(p);
            pull<P>(pl, g, xc, xcm, xcp, yl, o, Bf[(J + 2 + LEAD) % NBF]);
            Hh[(J + 2 + LEAD) % NBF] = halo_load(yl);
        }

        // Level 2, part 1: pre-collision populations at t+1 of row p - 2
        // (pulled from the ring rows p-3 .. p-1) and their psi.
        if (p >= 0) {
            // Formed here, collided two iterations later (which reads F2[J]).
            C(&Fr)[9] = F2[(J + 2) % NBF];
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                // f_i(x, t+1) = f*_i(x - c_i): lattice row y - c_y is walk
                // row r - c_y dir; lane l - c_x (clamped: lanes 0 and NT-1
                // form values no output uses).
                const int rr = p - 2 - q_cy(i) * dir;
                const int li = min(max(tid - q_cx(i), 0), NT - 1);
                Fr[i] = o.ld(&fs[(rr + 4) & 3][i][li], o.of(i));
            }
            ring2[slot2(4)][tid + 2] = psi_of(density(Fr), k2);
        }

        // Level 1: force and collision of row p into the ring of t+1.
        C anchor = (C)0;
        if (p <= nrows + 2) {
            auto slot = [&](int dy) {
                int v = s0 + 2 + dy * dir;
                return v >= RS ? v - RS : v;
            };
            const Stencil<C> st(ring[slot(-2)], ring[slot(-1)], ring[slot(0)], ring[slot(1)],
                                ring[slot(2)], tid + 2);
            C q[9];
            site_collide<false, P::kDev, kOm>(Bf[J % NBF], st, k, q, (C*)nullptr, o.o1, o.o2);
            S* lp[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) lp[i] = &fs[(p + 4) & 3][i][0];
            const uint32_t rnd = P::kDev ? site_hash(xc, wrow(p), k.step) : 0u;
            store_site<P>(lp, tid, q, o, rnd);
            anchor = q[1];
        }

        // Stage psi at t of row p + 3.
        {
            C(&NFr)[9] = Bf[(J + 3) % NBF];
            C& HF = Hh[(J + 3) % NBF];
#pragma unroll
            for (int i = 0; i < 9; ++i) asm volatile("" : "+v"(NFr[i]) : "v"(anchor));
            asm volatile("" : "+v"(HF) : "v"(anchor));
            int sl = s0 + 5;
            sl = sl >= RS ? sl - RS : sl;
            ring[sl][tid + 2] = psi_of(density(NFr), k);
            halo_psi(HF, sl);
        }
        __builtin_amdgcn_sched_barrier(0);
        __syncthreads();

        // Level 2, part 2: force and collision at t+1 of row q = p - 4, from
        // psi rows q-2 .. q+2 at t+1; store.
        const int qr = p - 4;
        if (qr >= 0 && qr < nrows) {
            // Walk rows are in walk order; psi row qr + dy (slot2(2 + dy)) is
            // lattice row ystart + (qr + dy) dir, i.e. the stencil's y + dy dir.
            const C* r_m2 = ring2[slot2(2 - 2 * dir)];
            const C* r_m1 = ring2[slot2(2 - dir)];
            const C* r_c = ring2[slot2(2)];
            const C* r_p1 = ring2[slot2(2 + dir)];
            const C* r_p2 = ring2[slot2(2 + 2 * dir)];
            const Stencil<C> st2(r_m2, r_m1, r_c, r_p1, r_p2, tid + 2);
            C q2[9];
            site_collide<false, P::kDev, kOm>(F2[J % NBF], st2, k2, q2, (C*)nullptr, o.o1, o.o2);
            if (own2) {
                const int yq = wrow(qr);
                const int xq = x0 + tid - 3;
                const uint32_t rnd = P::kDev ? site_hash(xq, yq, k2.step) : 0u;
                store_site<P>(pd, yq * g.pitch + xq, q2, o, rnd);
            }
        }
    };

    auto step_slot = [](int s) { return s + 1 >= RS ? s + 1 - RS : s + 1; };
    int s0 = 0;  // ring slot of level-1 walk row p - 2
    const int iters = nrows + 7;
#pragma unroll 1
    for (int it = 0;;) {
        group(Ic<0>{}, it, s0);
        s0 = step_slot(s0);
        if (++it >= iters) break;
        group(Ic<1>{}, it, s0);
        s0 = step_slot(s0);
        if (++it >= iters) break;
        group(Ic<2>{}, it, s0);
        s0 = step_slot(s0);
        if (++it >= iters) break;
        group(Ic<3>{}, it, s0);
        s0 = step_slot(s0);
        if (++it >= iters) break;
        if constexpr (NBF > 4) {
            group(Ic<4>{}, it, s0);
            s0 = step_slot(s0);
            if (++it >= iters) break;
        }
    }
}

template <class P, int NT>
__global__ void __launch_bounds__(NT)
k_step2(const typename P::S* __restrict__ src, typename P::S* __restrict__ dst, Geom g,
        CoefT<typename P::C> k)
{
    // tau = 1 (every run of the paper) and other tau as separate walks, so
    // the collision has no branch inside the loop.
    __shared__ Step2Smem<P, NT> sm;
    if (k.omega == (typename P::C)1)
        step2_tile<P, NT, 1>(src, dst, g, k, xcd_remap(blockIdx.x, gridDim.x), sm);
    else
        step2_tile<P, NT, 0>(src, dst, g, k, xcd_remap(blockIdx.x, gridDim.x), sm);
}

// One launch = one time step of one lattice: workgroup b updates logical
// tile xcd_remap(b).
template <class P, int NT, int MODE, int RPI, int LEAD>
__global__ void __launch_bounds__(NT)
k_step(const typename P::S* __restrict__ src, typename P::S* __restrict__ dst,
       Geom g, CoefT<typename P::C> k, double* __restrict__ partials)
{
    step_tile<P, NT, MODE, RPI, LEAD>(src, dst, g, k, partials, xcd_remap(blockIdx.x, gridDim.x));
}

// One launch = one time step of a batch of independent lattices.  The
// logical tiles of all lattices are numbered consecutively (lattice by
// lattice); tile_lattice maps a logical tile to its lattice, whose
// geometry, coefficients and buffers sit in desc.  Every lattice's tile is
// processed exactly as the single-lattice kernel processes it, so fields
// are bit-identical to single-lattice runs with the same tile shape.
template <class P, int NT>
__global__ void __launch_bounds__(NT)
k_step2_batch(const BatchLattice* __restrict__ desc, const int32_t* __restrict__ tile_lattice,
              int parity, uint32_t step)
{
    using S = typename P::S;
    const int gl = xcd_remap(blockIdx.x, gridDim.x);
    const int lat = tile_lattice[gl];
    const BatchLattice& d = desc[lat];
    static_assert(sizeof(typename P::C) == 4, "two-step kernels compute in single precision");
    const float* cf = d.coef_f;
    const CoefT<float> k{cf[0], cf[1], cf[2],  cf[3],  cf[4],  cf[5], cf[6],
                         cf[7], cf[8], cf[9], cf[10], cf[11], cf[12], step};
    __shared__ Step2Smem<P, NT> sm;  // tau = 1 and other tau as separate walks
    if (k.omega == 1.0f)
        step2_tile<P, NT, 1>(static_cast<const S*>(d.buf[parity]), static_cast<S*>(d.buf[parity ^ 1]),
                             d.geom2, k, gl - d.tile_begin2, sm);
    else
        step2_tile<P, NT, 0>(static_cast<const S*>(d.buf[parity]), static_cast<S*>(d.buf[parity ^ 1]),
                             d.geom2, k, gl - d.tile_begin2, sm);
}

template <class P, int NT, int MODE, int RPI, int LEAD>
__global__ void __launch_bounds__(NT)
k_step_batch(const BatchLattice* __restrict__ desc, const int32_t* __restrict__ tile_lattice,
             int parity, uint32_t step, double* __restrict__ partials)
{
    using S = typename P::S;
    const int gl = xcd_remap(blockIdx.x, gridDim.x);
    const int lat = tile_lattice[gl];
    const BatchLattice& d = desc[lat];
    CoefT<typename P::C> k = convert<typename P::C>(d.coef);
    k.step = step;
    step_tile<P, NT, MODE, RPI, LEAD>(static_cast<const S*>(d.buf[parity]),
                                static_cast<S*>(d.buf[parity ^ 1]), d.geom, k,
                                partials + (int64_t)d.tile_begin * 4, gl - d.tile_begin);
}

// Fixed-order reduction of the per-workgroup partials into one trace row
// {t, M, E_s, E_m, sum psi^2, E_bulk} (one workgroup of 256 threads).
__device__ __forceinline__ void final_row(const double* __restrict__ partials, int blocks,
                                          double t, double half_A1, double* __restrict__ out)
{
    __shared__ double sm[4][256];
    const int tid = threadIdx.x;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        double s = 0.0;
        for (int b = tid; b < blocks; b += 256) s += partials[(int64_t)b * 4 + q];
        sm[q][tid] = s;
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) {
#pragma unroll
            for (int q = 0; q < 4; ++q) sm[q][tid] += sm[q][tid + w];
        }
        __syncthreads();
    }
    if (tid == 0) {
        out[0] = t;
        out[1] = sm[0][0];
        out[2] = sm[1][0];
        out[3] = sm[2][0];
        out[4] = sm[3][0];
        out[5] = half_A1 * sm[3][0];
    }
}

__global__ void __launch_bounds__(256)
k_final(const double* __restrict__ partials, int blocks, double t, double half_A1,
        double* __restrict__ out)
{
    final_row(partials, blocks, t, half_A1, out);
}

// One workgroup per lattice of a batch: row `row` of each lattice's trace.
__global__ void __launch_bounds__(256)
k_final_batch(const BatchLattice* __restrict__ desc, const double* __restrict__ partials,
              double t, int64_t row)
{
    const BatchLattice& d = desc[blockIdx.x];
    final_row(partials + (int64_t)d.tile_begin * 4, d.geom.blocks, t, d.half_A1,
              d.trace + row * 6);
}

// rho and u = j / rho of the pre-collision state, dense [ny][nx] doubles.
template <class P>
__global__ void __launch_bounds__(256)
k_moments(const typename P::S* __restrict__ src, Geom g, typename P::C rho_ref,
          double* __restrict__ rho, double* __restrict__ ux, double* __restrict__ uy)
{
    using C = typename P::C;
    const int x = blockIdx.x * 256 + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= g.nx) return;
    const typename P::S* pl[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) pl[i] = src + (int64_t)i * g.plane;
    const Offs<P> o(rho_ref);
    C f[9];
    pull<P>(pl, g, x, x == 0 ? g.nx - 1 : x - 1, x == g.nx - 1 ? 0 : x + 1, y, o, f);
    const C r = density(f);
    const C jx = (f[1] - f[3]) + ((f[5] - f[7]) + (f[8] - f[6]));
    const C jy = (f[2] - f[4]) + ((f[5] - f[7]) + (f[6] - f[8]));
    const int64_t at = (int64_t)y * g.nx + x;
    if (rho) rho[at] = (double)r;
    if (ux) ux[at] = (double)jx / (double)r;
    if (uy) uy[at] = (double)jy / (double)r;
}

// Equilibrium populations f_i^eq(rho, u) of each site, stored upstream at
// x - c_i so that the next pull delivers them to x.
template <class P>
__global__ void __launch_bounds__(256)
k_init(const double* __restrict__ rho, const double* __restrict__ ux,
       const double* __restrict__ uy, typename P::S* __restrict__ dst, Geom g,
       typename P::C rho_ref)
{
    using C = typename P::C;
    const int x = blockIdx.x * 256 + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= g.nx) return;
    const int64_t at = (int64_t)y * g.nx + x;
    const C r = (C)rho[at];
    const C u = ux ? (C)ux[at] : (C)0;
    const C v = uy ? (C)uy[at] : (C)0;
    const C usq = (C)1.5 * (u * u + v * v);
    const Offs<P> o(rho_ref);
    const int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    const int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const C w = i == 0 ? (C)4 / (C)9 : (i < 5 ? (C)1 / (C)9 : (C)1 / (C)36);
        const C cu = (C)cx[i] * u + (C)cy[i] * v;
        const C feq = w * r * ((C)1 + (C)3 * cu + (C)4.5 * cu * cu - usq);
        const int xs = wrapi(x - cx[i], g.nx);
        const int ys = wrapi(y - cy[i], g.ny);
        P::st(dst + (int64_t)i * g.plane + (int64_t)ys * g.pitch + xs, feq, o.of(i));
    }
}

// Raw population words between the pitched upstream layout and a dense
// [9][ny][nx] array of pre-collision populations (an exact permutation).
template <typename W, bool kGet>
__global__ void __launch_bounds__(256)
k_state(const W* __restrict__ in, W* __restrict__ out, Geom g)
{
    const int x = blockIdx.x * 256 + threadIdx.x;
    const int y = blockIdx.y;
    const int i = blockIdx.z;
    if (x >= g.nx) return;
    const int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    const int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    const int64_t d = ((int64_t)i * g.ny + y) * g.nx + x;
    const int64_t s = (int64_t)i * g.plane + (int64_t)wrapi(y - cy[i], g.ny) * g.pitch +
                      wrapi(x - cx[i], g.nx);
    if (kGet)
        out[d] = in[s];
    else
        out[s] = in[d];
}

template <class P, int NT, int RPI>
hipError_t step_nt(int mode, const void* src, void* dst, const Geom& g,
                   const Coef& c, double* partials, hipStream_t s)
{
    using S = typename P::S;
    const auto k = convert<typename P::C>(c);
    const dim3 grid(g.blocks), block(NT);
    const S* a = static_cast<const S*>(src);
    S* b = static_cast<S*>(dst);
    if (mode == MODE_STEP) {
        if constexpr (lead2_variant<P, RPI>()) {
            if (g.tile_y >= kLead2MinRows) {
                hipLaunchKernelGGL((k_step<P, NT, MODE_STEP, RPI, 2>), grid, block, 0, s, a, b, g, k, partials);
                return hipGetLastError();
            }
        }
        hipLaunchKernelGGL((k_step<P, NT, MODE_STEP, RPI, 1>), grid, block, 0, s, a, b, g, k, partials);
    } else if (mode == MODE_STEP_ENERGY)
        hipLaunchKernelGGL((k_step<P, NT, MODE_STEP_ENERGY, RPI, 1>), grid, block, 0, s, a, b, g, k, partials);
    else if (mode == MODE_STEP_TAPE) {
        if constexpr (P::kDev)
            return hipErrorInvalidValue;
        else
            hipLaunchKernelGGL((k_step<P, NT, MODE_STEP_TAPE, RPI, 1>), grid, block, 0, s, a, b, g, k, partials);
    } else
        hipLaunchKernelGGL((k_step<P, NT, MODE_ENERGY, RPI, 1>), grid, block, 0, s, a, b, g, k, partials);
    return hipGetLastError();
}

template <class P, int NT>
hipError_t step2_nt(const void* src, void* dst, const Geom& g, const Coef& c, hipStream_t s)
{
    using S = typename P::S;
    const auto k = convert<typename P::C>(c);
    hipLaunchKernelGGL((k_step2<P, NT>), dim3(g.blocks), dim3(NT), 0, s, static_cast<const S*>(src),
                       static_cast<S*>(dst), g, k);
    return hipGetLastError();
}

template <class P, int NT>
hipError_t step_rpi(int mode, const void* src, void* dst, const Geom& g,
                    const Coef& c, double* partials, hipStream_t s)
{
    return g.rows_per_iter == 2 ? step_nt<P, NT, 2>(mode, src, dst, g, c, partials, s)
                                : step_nt<P, NT, 1>(mode, src, dst, g, c, partials, s);
}

template <class P>
hipError_t step_p(int mode, const void* src, void* dst, const Geom& g,
                  const Coef& c, double* partials, hipStream_t s)
{
    switch (g.tile_x) {
    case 64: return step_rpi<P, 64>(mode, src, dst, g, c, partials, s);
    case 128: return step_rpi<P, 128>(mode, src, dst, g, c, partials, s);
    case 256: return step_rpi<P, 256>(mode, src, dst, g, c, partials, s);
    default: return hipErrorInvalidValue;
    }
}

struct BatchLaunch {
    const BatchLattice* desc;
    const int32_t* tile_lattice;
    int tiles;
    int parity;
    uint32_t step;
    double* partials;
    int min_tile_y;  // smallest tile_y of the batch's lattices
};

template <class P, int NT, int RPI>
hipError_t batch_nt(int mode, const BatchLaunch& a, hipStream_t s)
{
    const dim3 grid(a.tiles), block(NT);
    if (mode == MODE_STEP) {
        if constexpr (lead2_variant<P, RPI>()) {
            if (a.min_tile_y >= kLead2MinRows) {
                hipLaunchKernelGGL((k_step_batch<P, NT, MODE_STEP, RPI, 2>), grid, block, 0, s, a.desc,
                                   a.tile_lattice, a.parity, a.step, a.partials);
                return hipGetLastError();
            }
        }
        hipLaunchKernelGGL((k_step_batch<P, NT, MODE_STEP, RPI, 1>), grid, block, 0, s, a.desc,
                           a.tile_lattice, a.parity, a.step, a.partials);
    } else if (mode == MODE_STEP_ENERGY)
        hipLaunchKernelGGL((k_step_batch<P, NT, MODE_STEP_ENERGY, RPI, 1>), grid, block, 0, s, a.desc,
                           a.tile_lattice, a.parity, a.step, a.partials);
    else
        hipLaunchKernelGGL((k_step_batch<P, NT, MODE_ENERGY, RPI, 1>), grid, block, 0, s, a.desc,
                           a.tile_lattice, a.parity, a.step, a.partials);
    return hipGetLastError();
}

template <class P>
hipError_t batch_p(int mode, int tile_x, int rpi, const BatchLaunch& a, hipStream_t s)
{
    const bool two = rpi == 2;
    switch (tile_x) {
    case 64: return two ? batch_nt<P, 64, 2>(mode, a, s) : batch_nt<P, 64, 1>(mode, a, s);
    case 128: return two ? batch_nt<P, 128, 2>(mode, a, s) : batch_nt<P, 128, 1>(mode, a, s);
    case 256: return two ? batch_nt<P, 256, 2>(mode, a, s) : batch_nt<P, 256, 1>(mode, a, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

template <class P>
hipError_t step2_p(const void* src, void* dst, const Geom& g, const Coef& c, hipStream_t s)
{
    switch (g.tile_x) {
    case 64: return step2_nt<P, 64>(src, dst, g, c, s);
    case 128: return step2_nt<P, 128>(src, dst, g, c, s);
    case 256: return step2_nt<P, 256>(src, dst, g, c, s);
    default: return hipErrorInvalidValue;
    }
}

template <class P>
hipError_t step2_batch_p(int tile_x, const BatchLattice* desc, const int32_t* tile_lattice,
                         int tiles, int parity, uint32_t step, hipStream_t s)
{
    const dim3 grid(tiles);
    switch (tile_x) {
    case 64:
        hipLaunchKernelGGL((k_step2_batch<P, 64>), grid, dim3(64), 0, s, desc, tile_lattice, parity, step);
        break;
    case 128:
        hipLaunchKernelGGL((k_step2_batch<P, 128>), grid, dim3(128), 0, s, desc, tile_lattice, parity, step);
        break;
    case 256:
        hipLaunchKernelGGL((k_step2_batch<P, 256>), grid, dim3(256), 0, s, desc, tile_lattice, parity, step);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_step2_batch(int storage, int tile_x, const BatchLattice* desc,
                              const int32_t* tile_lattice, int tiles, int parity, uint32_t step,
                              hipStream_t s)
{
    if (tiles <= 0) return hipErrorInvalidValue;
    switch (storage) {
    case ST_F32: return step2_batch_p<PF32>(tile_x, desc, tile_lattice, tiles, parity, step, s);
    case ST_F16DEV: return step2_batch_p<PF16>(tile_x, desc, tile_lattice, tiles, parity, step, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_step2(int storage, const void* src, void* dst, const Geom& g, const Coef& c,
                        hipStream_t s)
{
    switch (storage) {
    case ST_F32: return step2_p<PF32>(src, dst, g, c, s);
    case ST_F16DEV: return step2_p<PF16>(src, dst, g, c, s);
    default: return hipErrorInvalidValue;
    }
}

namespace {
template <class P>
const void* step2_kernel(int tile_x)
{
    switch (tile_x) {
    case 64: return reinterpret_cast<const void*>(k_step2<P, 64>);
    case 128: return reinterpret_cast<const void*>(k_step2<P, 128>);
    case 256: return reinterpret_cast<const void*>(k_step2<P, 256>);
    default: return nullptr;
    }
}
}  // namespace

int step2_resident(int storage, int tile_x)
{
    static std::mutex mu;
    static std::map<std::tuple<int, int, int>, int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return -1;
    const auto key = std::make_tuple(dev, storage, tile_x);
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    const void* fn = storage == ST_F32 ? step2_kernel<PF32>(tile_x)
                   : storage == ST_F16DEV ? step2_kernel<PF16>(tile_x) : nullptr;
    int cus = 0, per_cu = 0;
    if (!fn || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, tile_x, 0) != hipSuccess) {
        (void)hipGetLastError();
        return -1;
    }
    const int r = cus > 0 && per_cu > 0 ? cus * per_cu : -1;
    cache.emplace(key, r);
    return r;
}

hipError_t launch_step_batch(int storage, int mode, int tile_x, int rows_per_iter, int min_tile_y,
                             const BatchLattice* desc, const int32_t* tile_lattice, int tiles,
                             int parity, uint32_t step, double* partials, hipStream_t s)
{
    const BatchLaunch a{desc, tile_lattice, tiles, parity, step, partials, min_tile_y};
    switch (storage) {
    case ST_F64: return batch_p<PF64>(mode, tile_x, rows_per_iter, a, s);
    case ST_F32: return batch_p<PF32>(mode, tile_x, rows_per_iter, a, s);
    case ST_F16DEV: return batch_p<PF16>(mode, tile_x, rows_per_iter, a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_final_batch(const BatchLattice* desc, int count, const double* partials,
                              double t, int64_t row, hipStream_t s)
{
    hipLaunchKernelGGL(k_final_batch, dim3(count), dim3(256), 0, s, desc, partials, t, row);
    return hipGetLastError();
}

hipError_t launch_step(int storage, int mode, const void* src, void* dst,
                       const Geom& g, const Coef& c, double* partials,
                       hipStream_t s)
{
    switch (storage) {
    case ST_F64: return step_p<PF64>(mode, src, dst, g, c, partials, s);
    case ST_F32: return step_p<PF32>(mode, src, dst, g, c, partials, s);
    case ST_F16DEV: return step_p<PF16>(mode, src, dst, g, c, partials, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_final(const double* partials, int blocks, double t,
                        double half_A1, double* out_row, hipStream_t s)
{
    hipLaunchKernelGGL(k_final, dim3(1), dim3(256), 0, s, partials, blocks, t, half_A1, out_row);
    return hipGetLastError();
}

hipError_t launch_moments(int storage, const void* src, const Geom& g,
                          const Coef& c, double* rho, double* ux, double* uy,
                          hipStream_t s)
{
    const dim3 grid((g.nx + 255) / 256, g.ny), block(256);
    switch (storage) {
    case ST_F64:
        hipLaunchKernelGGL(k_moments<PF64>, grid, block, 0, s, static_cast<const double*>(src), g,
                           c.rho_ref, rho, ux, uy);
        break;
    case ST_F32:
        hipLaunchKernelGGL(k_moments<PF32>, grid, block, 0, s, static_cast<const float*>(src), g,
                           (float)c.rho_ref, rho, ux, uy);
        break;
    case ST_F16DEV:
        hipLaunchKernelGGL(k_moments<PF16>, grid, block, 0, s, static_cast<const _Float16*>(src), g,
                           (float)c.rho_ref, rho, ux, uy);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_init(int storage, const double* rho, const double* ux,
                       const double* uy, void* dst, const Geom& g,
                       const Coef& c, hipStream_t s)
{
    const dim3 grid((g.nx + 255) / 256, g.ny), block(256);
    switch (storage) {
    case ST_F64:
        hipLaunchKernelGGL(k_init<PF64>, grid, block, 0, s, rho, ux, uy, static_cast<double*>(dst), g,
                           c.rho_ref);
        break;
    case ST_F32:
        hipLaunchKernelGGL(k_init<PF32>, grid, block, 0, s, rho, ux, uy, static_cast<float*>(dst), g,
                           (float)c.rho_ref);
        break;
    case ST_F16DEV:
        hipLaunchKernelGGL(k_init<PF16>, grid, block, 0, s, rho, ux, uy, static_cast<_Float16*>(dst), g,
                           (float)c.rho_ref);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <bool kGet>
static hipError_t state_copy(int storage, const void* in, void* out, const Geom& g, hipStream_t s)
{
    const dim3 grid((g.nx + 255) / 256, g.ny, 9), block(256);
    switch (storage_bytes(storage)) {
    case 8:
        hipLaunchKernelGGL((k_state<uint64_t, kGet>), grid, block, 0, s,
                           static_cast<const uint64_t*>(in), static_cast<uint64_t*>(out), g);
        break;
    case 4:
        hipLaunchKernelGGL((k_state<uint32_t, kGet>), grid, block, 0, s,
                           static_cast<const uint32_t*>(in), static_cast<uint32_t*>(out), g);
        break;
    case 2:
        hipLaunchKernelGGL((k_state<uint16_t, kGet>), grid, block, 0, s,
                           static_cast<const uint16_t*>(in), static_cast<uint16_t*>(out), g);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_get_state(int storage, const void* src, void* dense, const Geom& g, hipStream_t s)
{
    return state_copy<true>(storage, src, dense, g, s);
}

hipError_t launch_set_state(int storage, const void* dense, void* dst, const Geom& g, hipStream_t s)
{
    return state_copy<false>(storage, dense, dst, g, s);
}

void coef_to_f32(const Coef& c, float out[13])
{
    const CoefT<float> k = convert<float>(c);
    const float v[13] = {k.K1, k.K2, k.K4, k.K5, k.K8, k.KE0, k.tau, k.omega,
                         k.sqrt_rho0, k.inv_rho0, k.rho_ref, k.K4x2, k.K8x2};
    for (int i = 0; i < 13; ++i) out[i] = v[i];
}

}  // namespace lbk
