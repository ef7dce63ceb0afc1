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
// Half-precision deviation from the rest-state equilibrium w_i rho_ref.
struct PF16 {
    using S = _Float16;
    using C = float;
    static constexpr bool kDev = true;
    __device__ static C ld(const S* p, C off) { return off + (C)(*p); }
    __device__ static void st(S* p, C v, C off) { *p = (S)(v - off); }
};

template <typename C>
struct CoefT {
    C K1, K2, K4, K5, K8, KE0, tau, omega, sqrt_rho0, inv_rho0, rho_ref;
};

template <typename C>
CoefT<C> convert(const Coef& c)
{
    return CoefT<C>{(C)c.K1, (C)c.K2, (C)c.K4, (C)c.K5, (C)c.K8, (C)c.KE0,
                    (C)c.tau, (C)c.omega, (C)c.sqrt_rho0, (C)c.inv_rho0,
                    (C)c.rho_ref};
}

__device__ __forceinline__ double exp_c(double v) { return exp(v); }
__device__ __forceinline__ float exp_c(float v) { return expf(v); }

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

// Deviation offsets w_i rho_ref of the half storage (zero otherwise).
template <class P>
struct Offs {
    typename P::C o0, o1, o2;  // rest, axis, diagonal
    __device__ Offs(typename P::C rho_ref)
    {
        using C = typename P::C;
        if (P::kDev) {
            o0 = rho_ref * ((C)4 / (C)9);
            o1 = rho_ref * ((C)1 / (C)9);
            o2 = rho_ref * ((C)1 / (C)36);
        } else {
            o0 = o1 = o2 = (C)0;
        }
    }
    __device__ typename P::C of(int i) const { return i == 0 ? o0 : (i < 5 ? o1 : o2); }
};

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
    const int64_t r0 = (int64_t)y * g.pitch, rm = (int64_t)ym * g.pitch,
                  rp = (int64_t)yp * g.pitch;
    f[0] = P::ld(pl[0] + r0 + x, o.o0);
    f[1] = P::ld(pl[1] + r0 + xm, o.o1);  // c = ( 1, 0)
    f[2] = P::ld(pl[2] + rm + x, o.o1);   // c = ( 0, 1)
    f[3] = P::ld(pl[3] + r0 + xp, o.o1);  // c = (-1, 0)
    f[4] = P::ld(pl[4] + rp + x, o.o1);   // c = ( 0,-1)
    f[5] = P::ld(pl[5] + rm + xm, o.o2);  // c = ( 1, 1)
    f[6] = P::ld(pl[6] + rm + xp, o.o2);  // c = (-1, 1)
    f[7] = P::ld(pl[7] + rp + xp, o.o2);  // c = (-1,-1)
    f[8] = P::ld(pl[8] + rp + xm, o.o2);  // c = ( 1,-1)
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
template <class P, int NT, int MODE>
__global__ void __launch_bounds__(NT)
k_step(const typename P::S* __restrict__ src, typename P::S* __restrict__ dst,
       Geom g, CoefT<typename P::C> k, double* __restrict__ partials)
{
    using S = typename P::S;
    using C = typename P::C;
    constexpr bool kEnergy = MODE != MODE_STEP;
    constexpr bool kCollide = MODE != MODE_ENERGY;
    constexpr int LW = NT + 4;
    __shared__ C ring[6][LW];

    const int tid = threadIdx.x;
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int sx = lb % g.tiles_x;
    const int sy = lb / g.tiles_x;
    const int x0 = sx * NT;
    const int y0 = sy * g.tile_y;
    const int y1 = min(y0 + g.tile_y, g.ny);
    const int nx = g.nx;

    const S* pl[9];
    S* pd[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        pl[i] = src + (int64_t)i * g.plane;
        pd[i] = dst + (int64_t)i * g.plane;
    }
    const Offs<P> o(k.rho_ref);

    // This lane's column (LDS column tid + 2) ...
    const bool own = x0 + tid < nx;
    const int xc = (x0 + tid) % nx;
    const int xcm = xc == 0 ? nx - 1 : xc - 1;
    const int xcp = xc == nx - 1 ? 0 : xc + 1;
    // ... and, for lanes 0..3, one halo column: LDS 0, 1, NT+2, NT+3.
    const bool halo = tid < 4;
    const int hc = tid < 2 ? tid : NT + tid;
    int hx = (x0 - 2 + hc) % nx;
    hx = hx < 0 ? hx + nx : hx;
    const int hxm = hx == 0 ? nx - 1 : hx - 1;
    const int hxp = hx == nx - 1 ? 0 : hx + 1;

    C R0[9], R1[9], L[9];

    // Prologue: psi of rows y0-2 .. y0+1 into ring slots 0..3; keep the
    // populations of rows y0 and y0+1.
#pragma unroll 1
    for (int j = -2; j < 2; ++j) {
        const int y = wrapi(y0 + j, g.ny);
        pull<P>(pl, g, xc, xcm, xcp, y, o, L);
        ring[j + 2][tid + 2] = psi_of(density(L), k);
        if (halo) {
            C h[9];
            pull<P>(pl, g, hx, hxm, hxp, y, o, h);
            ring[j + 2][hc] = psi_of(density(h), k);
        }
        if (j == 0) {
#pragma unroll
            for (int i = 0; i < 9; ++i) R0[i] = L[i];
        } else if (j == 1) {
#pragma unroll
            for (int i = 0; i < 9; ++i) R1[i] = L[i];
        }
    }

    double aM = 0.0, aEs = 0.0, aEm = 0.0, aS2 = 0.0;
    int s0 = 0;  // ring slot of row y - 2

#pragma unroll 1
    for (int y = y0; y < y1; ++y) {
        // Lead row y + 2 into slot s0 + 4.
        const int yl = wrapi(y + 2, g.ny);
        const int sl = s0 + 4 >= 6 ? s0 - 2 : s0 + 4;
        pull<P>(pl, g, xc, xcm, xcp, yl, o, L);
        ring[sl][tid + 2] = psi_of(density(L), k);
        if (halo) {
            C h[9];
            pull<P>(pl, g, hx, hxm, hxp, yl, o, h);
            ring[sl][hc] = psi_of(density(h), k);
        }
        __syncthreads();

        const int s1 = s0 + 1 >= 6 ? s0 - 5 : s0 + 1;
        const int s2 = s0 + 2 >= 6 ? s0 - 4 : s0 + 2;
        const int s3 = s0 + 3 >= 6 ? s0 - 3 : s0 + 3;
        const C* rm2 = ring[s0];
        const C* rm1 = ring[s1];
        const C* rc = ring[s2];
        const C* rp1 = ring[s3];
        const C* rp2 = ring[sl];
        const int c = tid + 2;

        const C p = rc[c];
        // psi(x + dx, y + dy), named by direction.
        const C e1 = rc[c + 1], w1 = rc[c - 1], n1 = rp1[c], s1v = rm1[c];
        const C ne = rp1[c + 1], nw = rp1[c - 1], sw = rm1[c - 1], se = rm1[c + 1];
        const C e2 = rc[c + 2], w2 = rc[c - 2], n2 = rp2[c], s2v = rm2[c];
        const C e2n = rp1[c + 2], e2s = rm1[c + 2], w2n = rp1[c - 2], w2s = rm1[c - 2];
        const C n2e = rp2[c + 1], n2w = rp2[c - 1], s2e = rm2[c + 1], s2w = rm2[c - 1];
        const C ne2 = rp2[c + 2], nw2 = rp2[c - 2], sw2 = rm2[c - 2], se2 = rm2[c + 2];

        if (kEnergy && own) {
            const C S1 = (e1 + w1) + (n1 + s1v);
            const C S2 = (ne + sw) + (nw + se);
            const C S4 = (e2 + w2) + (n2 + s2v);
            const C S5 = ((e2n + w2s) + (e2s + w2n)) + ((n2e + s2w) + (n2w + s2e));
            const C S8 = (ne2 + sw2) + (nw2 + se2);
            const C es = (C)0.5 * p * (k.KE0 * p + k.K1 * S1 + k.K2 * S2);
            const C em = (C)0.5 * p * (k.K4 * S4 + k.K5 * S5 + k.K8 * S8);
            aM += (double)density(R0);
            aEs += (double)es;
            aEm += (double)em;
            aS2 += (double)p * (double)p;
        }

        if (kCollide) {
            // eq. (FORCE): F = -psi(x) sum_k K_k psi(x + c_k) c_k, links
            // paired with their opposites.
            const C sumx = k.K1 * (e1 - w1) + k.K2 * ((ne + se) - (nw + sw)) +
                           (C)2 * k.K4 * (e2 - w2) +
                           k.K5 * ((C)2 * ((e2n + e2s) - (w2n + w2s)) + ((n2e + s2e) - (n2w + s2w))) +
                           (C)2 * k.K8 * ((ne2 + se2) - (nw2 + sw2));
            const C sumy = k.K1 * (n1 - s1v) + k.K2 * ((ne + nw) - (se + sw)) +
                           (C)2 * k.K4 * (n2 - s2v) +
                           k.K5 * ((C)2 * ((n2e + n2w) - (s2e + s2w)) + ((e2n + w2n) - (e2s + w2s))) +
                           (C)2 * k.K8 * ((ne2 + nw2) - (se2 + sw2));
            const C Fx = -p * sumx;
            const C Fy = -p * sumy;

            // BGK collision at u_eq = (j + tau F) / rho.
            const C rho = density(R0);
            const C jx = (R0[1] - R0[3]) + ((R0[5] - R0[7]) + (R0[8] - R0[6]));
            const C jy = (R0[2] - R0[4]) + ((R0[5] - R0[7]) + (R0[6] - R0[8]));
            const C inv = (C)1 / rho;
            const C ux = (jx + k.tau * Fx) * inv;
            const C uy = (jy + k.tau * Fy) * inv;
            const C usq = (C)1.5 * (ux * ux + uy * uy);
            const C r1 = rho * ((C)1 / (C)9);
            const C r2 = rho * ((C)1 / (C)36);
            const C om = k.omega;
            C q[9];
            auto axis = [&](C cu) { return r1 * ((C)1 + (C)3 * cu + (C)4.5 * cu * cu - usq); };
            auto diag = [&](C cu) { return r2 * ((C)1 + (C)3 * cu + (C)4.5 * cu * cu - usq); };
            q[1] = R0[1] + om * (axis(ux) - R0[1]);
            q[2] = R0[2] + om * (axis(uy) - R0[2]);
            q[3] = R0[3] + om * (axis(-ux) - R0[3]);
            q[4] = R0[4] + om * (axis(-uy) - R0[4]);
            q[5] = R0[5] + om * (diag(ux + uy) - R0[5]);
            q[6] = R0[6] + om * (diag(uy - ux) - R0[6]);
            q[7] = R0[7] + om * (diag(-ux - uy) - R0[7]);
            q[8] = R0[8] + om * (diag(ux - uy) - R0[8]);
            // The collision conserves mass exactly; take the rest
            // population from that so rounding cannot drift the mass.
            q[0] = rho - (((q[1] + q[3]) + (q[2] + q[4])) + ((q[5] + q[7]) + (q[6] + q[8])));
            if (own) {
                const int64_t at = (int64_t)y * g.pitch + xc;
#pragma unroll
                for (int i = 0; i < 9; ++i) P::st(pd[i] + at, q[i], o.of(i));
            }
        }

#pragma unroll
        for (int i = 0; i < 9; ++i) {
            R0[i] = R1[i];
            R1[i] = L[i];
        }
        s0 = s1;
    }

    if (kEnergy) {
        __shared__ double red[4][NT / 64];
        double v[4] = {aM, aEs, aEm, aS2};
        const int lane = tid & 63, wid = tid >> 6;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            v[q] = wave_sum(v[q]);
            if (lane == 0) red[q][wid] = v[q];
        }
        __syncthreads();
        if (tid < 4) {
            double s = 0.0;
            for (int w = 0; w < NT / 64; ++w) s += red[tid][w];
            partials[(int64_t)lb * 4 + tid] = s;
        }
    }
}

// Fixed-order reduction of the per-workgroup partials into one trace row
// {t, M, E_s, E_m, sum psi^2, E_bulk}.
__global__ void __launch_bounds__(256)
k_final(const double* __restrict__ partials, int blocks, double t,
        double half_A1, double* __restrict__ out)
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

template <class P, int NT>
hipError_t step_nt(int mode, const void* src, void* dst, const Geom& g,
                   const Coef& c, double* partials, hipStream_t s)
{
    using S = typename P::S;
    const auto k = convert<typename P::C>(c);
    const dim3 grid(g.blocks), block(NT);
    const S* a = static_cast<const S*>(src);
    S* b = static_cast<S*>(dst);
    if (mode == MODE_STEP)
        hipLaunchKernelGGL((k_step<P, NT, MODE_STEP>), grid, block, 0, s, a, b, g, k, partials);
    else if (mode == MODE_STEP_ENERGY)
        hipLaunchKernelGGL((k_step<P, NT, MODE_STEP_ENERGY>), grid, block, 0, s, a, b, g, k, partials);
    else
        hipLaunchKernelGGL((k_step<P, NT, MODE_ENERGY>), grid, block, 0, s, a, b, g, k, partials);
    return hipGetLastError();
}

template <class P>
hipError_t step_p(int mode, const void* src, void* dst, const Geom& g,
                  const Coef& c, double* partials, hipStream_t s)
{
    switch (g.tile_x) {
    case 64: return step_nt<P, 64>(mode, src, dst, g, c, partials, s);
    case 128: return step_nt<P, 128>(mode, src, dst, g, c, partials, s);
    case 256: return step_nt<P, 256>(mode, src, dst, g, c, partials, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

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

}  // namespace lbk
