// Adjoint (reverse-mode) kernels of the two-belt Shan-Chen step, for the
// gradients of a functional of the state at time T with respect to G1, G2
// and the initial density.
//
// Forward step at a site x (section II moments, eq. (FORCE), velocity-shift
// BGK collision, streaming of eq. (1)):
//   rho = sum f, j = sum c f, psi = sqrt(rho0) (1 - exp(-rho/rho0)),
//   F = -psi(x) S(x), S(x) = sum_k K_k psi(x + c_k) c_k, u = (j + tau F)/rho,
//   f*_l = f_l + w (feq_l(rho, u) - f_l), f_l(x + c_l, t+1) = f*_l(x),
//   feq_l = w_l rho phi_l(u), phi_l = 1 + 3 c_l.u + 4.5 (c_l.u)^2 - 1.5 u^2.
// Write lambda_i(x, t) = dL/df_i(x, t) (pre-collision populations).  The
// transpose of the pull streaming hands each site the adjoint of its
// post-collision populations, mu_l(x) = lambda_l(x + c_l, t+1), taken here as
// a gather so that no two threads write one value.  With
//   M0 = sum_l mu_l w_l phi_l,  V = sum_l mu_l w_l grad_u phi_l,
//   grad_u phi_l = 3 c_l + 9 (c_l.u) c_l - 3 u,
// one adjoint step is
//   lambda_i(x, t) = (1 - w) mu_i + w (M0 - V.u) + w V.c_i + g_rho(x),
//   g_F(x) = w tau V                                (dL/dF(x)),
//   g_rho(y) = psi'(rho(y)) * (-sum_k K_k psi(y + c_k) (g_F(y) - g_F(y + c_k)).c_k),
//   dL/dG1 += sum_x g_F(x).(-psi(x) sum_{first belt} w_k psi(x + c_k) c_k),
//   dL/dG2 += sum_x g_F(x).(-psi(x) sum_k p_k psi(x + c_k) c_k),
// where the g_rho sum is the force's dependence on psi, transposed from the
// 24-link gather into a 24-link gather of g_F (K_{-k} = K_k).
//
// Storage: lambda is kept as lam_i(x) + g(x), the 9 planes `lam` without the
// site term and the field `g` = g_rho (a 10th value per site), so the site
// term is added while the next step gathers mu instead of in a separate
// read-modify-write of 9 planes.  Tape entries are (rho, jx, jy, psi) of the
// pre-collision state.  All arrays are dense [component][ny][nx].  Sums are
// per-workgroup FP64 partials combined in a fixed order (no atomics), so
// gradients are bit-reproducible.
#include "lb_internal.h"

#include <hip/hip_runtime.h>

namespace lbk {
namespace {

// The 24 links (first belt in D2Q9 order, then |c|^2 = 4, 5, 8), the D2Q9
// weight of the first-belt links (0 on the second belt) and the Table 1
// weight p(|c|^2) of every link: K_k = G1 w_k + G2 p_k.
constexpr int kLx[24] = {1, 0, -1, 0, 1, -1, -1, 1, 2, 0, -2, 0,
                         2, 1, -1, -2, -2, -1, 1, 2, 2, -2, -2, 2};
constexpr int kLy[24] = {0, 1, 0, -1, 1, 1, -1, -1, 0, 2, 0, -2,
                         1, 2, 2, 1, -1, -2, -2, -1, 2, 2, -2, -2};
constexpr double kLw[24] = {1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                            0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
constexpr double kLp[24] = {4.0 / 63, 4.0 / 63, 4.0 / 63, 4.0 / 63,
                            4.0 / 135, 4.0 / 135, 4.0 / 135, 4.0 / 135,
                            1.0 / 180, 1.0 / 180, 1.0 / 180, 1.0 / 180,
                            2.0 / 945, 2.0 / 945, 2.0 / 945, 2.0 / 945,
                            2.0 / 945, 2.0 / 945, 2.0 / 945, 2.0 / 945,
                            1.0 / 15120, 1.0 / 15120, 1.0 / 15120, 1.0 / 15120};
// D2Q9 speeds and weights.
constexpr int kQx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int kQy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr double kQw[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                           1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
// Rest weights of E_s: w_0 and p_s0 = 247/420.
constexpr double kW0 = 4.0 / 9.0, kPS0 = 247.0 / 420.0;

constexpr int kThreads = 256;

__device__ __forceinline__ int wrapn(int v, int n)
{
    v = v < 0 ? v + n : v;
    return v >= n ? v - n : v;
}

// Site s of the dense [ny][nx] arrays with the offsets of rows y-2 .. y+2
// and the columns x-2 .. x+2, wrapped periodically, so that the element of
// neighbour (dx, dy) is at(dx, dy).  Element offsets fit in 32 bits and
// byte offsets too (the host limits an adjoint lattice to 2^29 sites).
struct Nbhd {
    int x, y, ro[5], cx[5];
    __device__ __forceinline__ Nbhd(int s, int nx, int ny)
    {
        const int N = nx * ny;
        y = (int)((unsigned)s / (unsigned)nx);
        x = s - y * nx;
        ro[2] = s - x;
        ro[3] = ro[2] + nx;
        ro[3] = ro[3] >= N ? ro[3] - N : ro[3];
        ro[4] = ro[3] + nx;
        ro[4] = ro[4] >= N ? ro[4] - N : ro[4];
        ro[1] = ro[2] - nx;
        ro[1] = ro[1] < 0 ? ro[1] + N : ro[1];
        ro[0] = ro[1] - nx;
        ro[0] = ro[0] < 0 ? ro[0] + N : ro[0];
#pragma unroll
        for (int k = 0; k < 5; ++k) cx[k] = wrapn(x + k - 2, nx);
    }
    __device__ __forceinline__ int at(int dx, int dy) const { return ro[dy + 2] + cx[dx + 2]; }
};

// base[e] with the byte offset formed in 32 bits (a uniform base plus a
// per-lane 32-bit offset, which needs no 64-bit address arithmetic).
template <typename T>
__device__ __forceinline__ T ld32(const T* base, int e)
{
    const uint32_t b = (uint32_t)e * (uint32_t)sizeof(T);
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + b);
}

__device__ __forceinline__ double ex(double v) { return exp(v); }
__device__ __forceinline__ float ex(float v) { return expf(v); }
__device__ __forceinline__ double sq(double v) { return sqrt(v); }
__device__ __forceinline__ float sq(float v) { return sqrtf(v); }

template <typename C>
struct AdjArgs {
    int nx, ny;
    int64_t N;
    C G1, G2, tau, omega, sqrt_rho0, inv_rho0;
};

// Workgroup sums of NV values, written (add = false) or added (add = true)
// to part[block * NV + v]; repeated launches of one grid therefore
// accumulate in a fixed order.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* __restrict__ part, bool add)
{
    __shared__ double red[NV][kThreads / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double s = v[q];
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) s += __shfl_xor(s, m, 64);
        if (lane == 0) red[q][wid] = s;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        const int q = threadIdx.x;
        const double s = (red[q][0] + red[q][1]) + (red[q][2] + red[q][3]);
        double* slot = part + (int64_t)blockIdx.x * NV + q;
        *slot = add ? *slot + s : s;
    }
}

// Tape entry of the pre-collision state held (as post-collision values of
// the previous step) in a pitched population buffer: rho, jx, jy, psi.
template <typename S, typename C>
__global__ void __launch_bounds__(kThreads)
k_adj_tape(const S* __restrict__ st, Geom g, AdjArgs<C> a, C* __restrict__ tape)
{
    const int64_t s = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (s >= a.N) return;
    const int x = (int)(s % a.nx), y = (int)(s / a.nx);
    C r = 0, jx = 0, jy = 0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int xs = wrapn(x - kQx[i], a.nx), ys = wrapn(y - kQy[i], a.ny);
        const C f = (C)st[(int64_t)i * g.plane + (int64_t)ys * g.pitch + xs];
        r += f;
        if (kQx[i]) jx += kQx[i] > 0 ? f : -f;
        if (kQy[i]) jy += kQy[i] > 0 ? f : -f;
    }
    tape[s] = r;
    tape[a.N + s] = jx;
    tape[2 * a.N + s] = jy;
    tape[3 * a.N + s] = a.sqrt_rho0 * ((C)1 - ex(-r * a.inv_rho0));
}

// First pass of one adjoint step: the local collision adjoint, g_F and the
// step's dL/dG1, dL/dG2 terms (added to the per-workgroup partials).
template <typename C>
__global__ void __launch_bounds__(kThreads)
k_adj_a(const C* __restrict__ lam_next, const C* __restrict__ g_next, const C* __restrict__ tape,
        AdjArgs<C> a, C* __restrict__ lam, C* __restrict__ gF, double* __restrict__ part)
{
    const int s = blockIdx.x * kThreads + threadIdx.x;
    double dg[2] = {0.0, 0.0};
    if (s < a.N) {
        const Nbhd nb(s, a.nx, a.ny);
        const C* psi = tape + 3 * a.N;
        C mu[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const int n = nb.at(kQx[i], kQy[i]);
            mu[i] = ld32(lam_next + i * a.N, n) + ld32(g_next, n);
        }
        const C rho = ld32(tape, s), jx = ld32(tape + a.N, s), jy = ld32(tape + 2 * a.N, s),
                p = ld32(psi, s);
        C s1x = 0, s1y = 0, s2x = 0, s2y = 0;
#pragma unroll
        for (int k = 0; k < 24; ++k) {
            const C pn = ld32(psi, nb.at(kLx[k], kLy[k]));
            if (k < 8) {
                s1x += (C)(kLw[k] * kLx[k]) * pn;
                s1y += (C)(kLw[k] * kLy[k]) * pn;
            }
            s2x += (C)(kLp[k] * kLx[k]) * pn;
            s2y += (C)(kLp[k] * kLy[k]) * pn;
        }
        // F = -psi (G1 s1 + G2 s2): the two belts' sums, weighted.
        const C Fx = -p * (a.G1 * s1x + a.G2 * s2x), Fy = -p * (a.G1 * s1y + a.G2 * s2y);
        const C ux = (jx + a.tau * Fx) / rho, uy = (jy + a.tau * Fy) / rho;
        const C uu = ux * ux + uy * uy;
        C M0 = 0, Vx = 0, Vy = 0;
#pragma unroll
        for (int l = 0; l < 9; ++l) {
            const C cu = (C)kQx[l] * ux + (C)kQy[l] * uy;
            const C wm = (C)kQw[l] * mu[l];
            M0 += wm * ((C)1 + (C)3 * cu + (C)4.5 * cu * cu - (C)1.5 * uu);
            Vx += wm * ((C)(3 * kQx[l]) + (C)9 * cu * (C)kQx[l] - (C)3 * ux);
            Vy += wm * ((C)(3 * kQy[l]) + (C)9 * cu * (C)kQy[l] - (C)3 * uy);
        }
        const C om = a.omega;
        const C base = om * (M0 - (Vx * ux + Vy * uy));
#pragma unroll
        for (int i = 0; i < 9; ++i)
            lam[i * a.N + s] = ((C)1 - om) * mu[i] + base + om * ((C)kQx[i] * Vx + (C)kQy[i] * Vy);
        const C gx = om * a.tau * Vx, gy = om * a.tau * Vy;
        gF[s] = gx;
        gF[a.N + s] = gy;
        dg[0] = -(double)p * ((double)gx * (double)s1x + (double)gy * (double)s1y);
        dg[1] = -(double)p * ((double)gx * (double)s2x + (double)gy * (double)s2y);
    }
    block_sum<2>(dg, part, true);
}

// Second pass: g_rho of every site, a 24-link gather of g_F.
template <typename C>
__global__ void __launch_bounds__(kThreads)
k_adj_b(const C* __restrict__ tape, const C* __restrict__ gF, AdjArgs<C> a, C* __restrict__ g)
{
    const int s = blockIdx.x * kThreads + threadIdx.x;
    if (s >= a.N) return;
    const Nbhd nb(s, a.nx, a.ny);
    const C* psi = tape + 3 * a.N;
    const C* gFy = gF + a.N;
    const C gx = ld32(gF, s), gy = ld32(gFy, s);
    C acc = 0;
#pragma unroll
    for (int k = 0; k < 24; ++k) {
        const int n = nb.at(kLx[k], kLy[k]);
        const C Kk = a.G1 * (C)kLw[k] + a.G2 * (C)kLp[k];
        acc += Kk * ld32(psi, n) * ((gx - ld32(gF, n)) * (C)kLx[k] + (gy - ld32(gFy, n)) * (C)kLy[k]);
    }
    // psi' = exp(-rho/rho0) sqrt(rho0)/rho0 = (sqrt(rho0) - psi)/rho0.
    g[s] = -acc * ((a.sqrt_rho0 - ld32(psi, s)) * a.inv_rho0);
}

// Interface measure: a(x) = sqrt(Dx^2 + Dy^2 + eps^2) from central
// differences of rho; stores (Dx/a, Dy/a) and the workgroup sums of a.
template <typename C>
__global__ void __launch_bounds__(kThreads)
k_adj_area(const C* __restrict__ tape, AdjArgs<C> a, C eps, C* __restrict__ dir,
           double* __restrict__ part)
{
    const int64_t s = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    double v[1] = {0.0};
    if (s < a.N) {
        const int x = (int)(s % a.nx), y = (int)(s / a.nx);
        const int64_t row = (int64_t)y * a.nx;
        const C dx = (C)0.5 * (tape[row + wrapn(x + 1, a.nx)] - tape[row + wrapn(x - 1, a.nx)]);
        const C dy = (C)0.5 * (tape[(int64_t)wrapn(y + 1, a.ny) * a.nx + x] -
                               tape[(int64_t)wrapn(y - 1, a.ny) * a.nx + x]);
        const C len = sq(dx * dx + dy * dy + eps * eps);
        dir[s] = dx / len;
        dir[a.N + s] = dy / len;
        v[0] = (double)len;
    }
    block_sum<1>(v, part, false);
}

// Seed at T: lambda_i(x, T) = dL/drho(x) for every i (held as lam = 0 and
// g = dL/drho), with dL/drho = 2 (E - E*) dE/dpsi psi' + beta dA/drho,
// dE/dpsi(x) = KE_0 psi(x) + sum_k K_k psi(x + c_k); also the workgroup sums
// of dE/dG1 = 1/2 sum psi (w_0 psi + sum w_k psi_k) and dE/dG2 likewise with
// p_s0, p_k.
template <typename C>
__global__ void __launch_bounds__(kThreads)
k_adj_seed(const C* __restrict__ tape, const C* __restrict__ dir, AdjArgs<C> a, C two_dE, C beta,
           C* __restrict__ lam, C* __restrict__ g, double* __restrict__ part)
{
    const int64_t s = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    double v[2] = {0.0, 0.0};
    if (s < a.N) {
        const int x = (int)(s % a.nx), y = (int)(s / a.nx);
        const C* psi = tape + 3 * a.N;
        const C p = psi[s];
        C e1 = (C)kW0 * p, e2 = (C)kPS0 * p;
#pragma unroll
        for (int k = 0; k < 24; ++k) {
            const C pn = psi[(int64_t)wrapn(y + kLy[k], a.ny) * a.nx + wrapn(x + kLx[k], a.nx)];
            if (k < 8) e1 += (C)kLw[k] * pn;
            e2 += (C)kLp[k] * pn;
        }
        const int64_t row = (int64_t)y * a.nx;
        const C dA = (C)0.5 * ((dir[row + wrapn(x - 1, a.nx)] - dir[row + wrapn(x + 1, a.nx)]) +
                               (dir[a.N + (int64_t)wrapn(y - 1, a.ny) * a.nx + x] -
                                dir[a.N + (int64_t)wrapn(y + 1, a.ny) * a.nx + x]));
        const C dpsi = (a.sqrt_rho0 - p) * a.inv_rho0;
        g[s] = two_dE * (a.G1 * e1 + a.G2 * e2) * dpsi + beta * dA;
#pragma unroll
        for (int i = 0; i < 9; ++i) lam[i * a.N + s] = (C)0;
        v[0] = 0.5 * (double)p * (double)e1;
        v[1] = 0.5 * (double)p * (double)e2;
    }
    block_sum<2>(v, part, false);
}

// dL/drho_init(x) = sum_i w_i lambda_i(x, 0) (populations start at w_i rho).
template <typename C>
__global__ void __launch_bounds__(kThreads)
k_adj_rho_grad(const C* __restrict__ lam, const C* __restrict__ g, int64_t N, double* __restrict__ out)
{
    const int64_t s = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (s >= N) return;
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) acc += kQw[i] * (double)lam[i * N + s];
    out[s] = acc + (double)g[s];
}

// out[v] = sum_b part[b * nv + v], in a fixed order (one workgroup).
__global__ void __launch_bounds__(kThreads)
k_adj_reduce(const double* __restrict__ part, int blocks, int nv, double* __restrict__ out)
{
    __shared__ double sm[kThreads];
    for (int v = 0; v < nv; ++v) {
        double s = 0.0;
        for (int b = threadIdx.x; b < blocks; b += kThreads) s += part[(int64_t)b * nv + v];
        sm[threadIdx.x] = s;
        __syncthreads();
        for (int w = kThreads / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[v] = sm[0];
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kThreads) k_adj_zero(double* __restrict__ p, int64_t n)
{
    const int64_t s = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (s < n) p[s] = 0.0;
}

template <typename C>
AdjArgs<C> adj_args(const AdjParams& p)
{
    return AdjArgs<C>{p.nx, p.ny, (int64_t)p.nx * p.ny, (C)p.G1, (C)p.G2, (C)p.tau,
                      (C)(1.0 / p.tau), (C)p.sqrt_rho0, (C)p.inv_rho0};
}

dim3 grid_of(int64_t n) { return dim3((unsigned)((n + kThreads - 1) / kThreads)); }

template <typename C>
hipError_t step_t(const AdjParams& p, const void* lam_next, const void* g_next, const void* tape,
                  void* lam, void* g, void* gF, double* part, hipStream_t s)
{
    const AdjArgs<C> a = adj_args<C>(p);
    hipLaunchKernelGGL(k_adj_a<C>, grid_of(a.N), dim3(kThreads), 0, s,
                       static_cast<const C*>(lam_next), static_cast<const C*>(g_next),
                       static_cast<const C*>(tape), a, static_cast<C*>(lam), static_cast<C*>(gF),
                       part);
    hipLaunchKernelGGL(k_adj_b<C>, grid_of(a.N), dim3(kThreads), 0, s, static_cast<const C*>(tape),
                       static_cast<const C*>(gF), a, static_cast<C*>(g));
    return hipGetLastError();
}

template <typename C>
hipError_t seed_t(const AdjParams& p, const void* tape, const void* dir, double two_dE, double beta,
                  void* lam, void* g, double* part, hipStream_t s)
{
    const AdjArgs<C> a = adj_args<C>(p);
    hipLaunchKernelGGL(k_adj_seed<C>, grid_of(a.N), dim3(kThreads), 0, s,
                       static_cast<const C*>(tape), static_cast<const C*>(dir), a, (C)two_dE,
                       (C)beta, static_cast<C*>(lam), static_cast<C*>(g), part);
    return hipGetLastError();
}

}  // namespace

int adj_blocks(int64_t n) { return (int)((n + kThreads - 1) / kThreads); }

hipError_t adj_tape(int storage, const void* st, const Geom& geom, const AdjParams& p, void* tape,
                    hipStream_t s)
{
    const int64_t N = (int64_t)p.nx * p.ny;
    if (storage == ST_F64)
        hipLaunchKernelGGL((k_adj_tape<double, double>), grid_of(N), dim3(kThreads), 0, s,
                           static_cast<const double*>(st), geom, adj_args<double>(p),
                           static_cast<double*>(tape));
    else if (storage == ST_F32)
        hipLaunchKernelGGL((k_adj_tape<float, float>), grid_of(N), dim3(kThreads), 0, s,
                           static_cast<const float*>(st), geom, adj_args<float>(p),
                           static_cast<float*>(tape));
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t adj_step(const AdjParams& p, const void* lam_next, const void* g_next, const void* tape,
                    void* lam, void* g, void* gF, double* part, hipStream_t s)
{
    return p.f64 ? step_t<double>(p, lam_next, g_next, tape, lam, g, gF, part, s)
                 : step_t<float>(p, lam_next, g_next, tape, lam, g, gF, part, s);
}

hipError_t adj_area(const AdjParams& p, const void* tape, double eps, void* dir, double* part,
                    hipStream_t s)
{
    const int64_t N = (int64_t)p.nx * p.ny;
    if (p.f64)
        hipLaunchKernelGGL(k_adj_area<double>, grid_of(N), dim3(kThreads), 0, s,
                           static_cast<const double*>(tape), adj_args<double>(p), eps,
                           static_cast<double*>(dir), part);
    else
        hipLaunchKernelGGL(k_adj_area<float>, grid_of(N), dim3(kThreads), 0, s,
                           static_cast<const float*>(tape), adj_args<float>(p), (float)eps,
                           static_cast<float*>(dir), part);
    return hipGetLastError();
}

hipError_t adj_seed(const AdjParams& p, const void* tape, const void* dir, double two_dE, double beta,
                    void* lam, void* g, double* part, hipStream_t s)
{
    return p.f64 ? seed_t<double>(p, tape, dir, two_dE, beta, lam, g, part, s)
                 : seed_t<float>(p, tape, dir, two_dE, beta, lam, g, part, s);
}

hipError_t adj_rho_grad(const AdjParams& p, const void* lam, const void* g, double* out, hipStream_t s)
{
    const int64_t N = (int64_t)p.nx * p.ny;
    if (p.f64)
        hipLaunchKernelGGL(k_adj_rho_grad<double>, grid_of(N), dim3(kThreads), 0, s,
                           static_cast<const double*>(lam), static_cast<const double*>(g), N, out);
    else
        hipLaunchKernelGGL(k_adj_rho_grad<float>, grid_of(N), dim3(kThreads), 0, s,
                           static_cast<const float*>(lam), static_cast<const float*>(g), N, out);
    return hipGetLastError();
}

hipError_t adj_reduce(const double* part, int blocks, int nv, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_adj_reduce, dim3(1), dim3(kThreads), 0, s, part, blocks, nv, out);
    return hipGetLastError();
}

hipError_t adj_zero(double* p, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_adj_zero, grid_of(n), dim3(kThreads), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace lbk
