// Section V observables of a dense population array without a context or a
// workspace (lb_pseudo_energy_state in include/lb.h), for callers that
// cannot allocate device memory.
//
// The per-workgroup partial sums and the result row live in `scratch`, a
// file-scope device array of fixed size that every call on a GPU shares.
// Host code never passes the array's name to a kernel: its device address
// is looked up once per device (hipGetSymbolAddress, with that device
// current) and that address is what the kernels receive.
//
// Per site the arithmetic is the one the step kernel's energy pass does
// (same density association, psi, link sums and products, contraction off),
// so each site contributes the same value; only the order in which the
// double-precision site values are summed differs.
#include "lb_internal.h"

#include <hip/hip_runtime.h>

#include <mutex>

namespace lbk {
namespace {

constexpr int kNaBlocks = 1024;         // workgroups of a call = partials in scratch
constexpr int kNaTx = 64, kNaTy = 4;    // sites of a tile (one per thread)
constexpr int kNaThreads = kNaTx * kNaTy;
constexpr int kNaLx = kNaTx + 4, kNaLy = kNaTy + 4;  // tile plus the 2-site halo
constexpr int kNaScratchDoubles = kNaBlocks * 4 + 8;  // partials, then the row

}  // namespace
}  // namespace lbk

// kNaBlocks partial sums of {M, E_s, E_m, sum psi^2} and one result row
// {t, M, E_s, E_m, sum psi^2, E_bulk}: 32.8 KB per GPU.
static __device__ __align__(256) double scratch[lbk::kNaScratchDoubles];

namespace lbk {
namespace {

std::mutex g_na_mu;
constexpr int kNaMaxDevices = 64;
double* g_na_ptr[kNaMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once).
hipError_t scratch_ptr(double** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kNaMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_na_mu);
    if (!g_na_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_na_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_na_ptr[dev];
    return hipSuccess;
}

template <typename S, typename C>
struct NaCoef {
    C KE0, K1, K2, K4, K5, K8, sqrt_rho0, inv_rho0;
    C o0, o1, o2;  // deviation offsets w_i rho_ref (half storage), else 0
};

template <typename S, typename C>
__device__ __forceinline__ C na_ld(const S* p, C off)
{
#pragma clang fp contract(off)
    if constexpr (sizeof(S) == 2) {
        return off + (C)(*p);
    } else {
        return (C)(*p);
    }
}

__device__ __forceinline__ double na_exp(double v) { return exp(v); }
__device__ __forceinline__ float na_exp(float v) { return __expf(v); }

__device__ __forceinline__ int na_wrap(int v, int n)
{
    v = v < 0 ? v + n : v;
    return v >= n ? v - n : v;
}

__device__ __forceinline__ double na_wave_sum(double v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// Grid-stride over 64 x 4 tiles; every workgroup writes one partial of each
// sum.  Site values are accumulated in a fixed order, so results are
// reproducible.
template <typename S, typename C>
__global__ void __launch_bounds__(kNaThreads)
k_na_energy(const S* __restrict__ f, int nx, int ny, NaCoef<S, C> k, double* __restrict__ part)
{
#pragma clang fp contract(off)
    __shared__ C ps[kNaLy][kNaLx];
    __shared__ C rh[kNaTy][kNaTx];
    __shared__ double red[4][kNaThreads / 64];
    const int tid = threadIdx.x;
    const int tx = tid % kNaTx, ty = tid / kNaTx;
    const int tiles_x = (nx + kNaTx - 1) / kNaTx;
    const int tiles = tiles_x * ((ny + kNaTy - 1) / kNaTy);
    const int64_t N = (int64_t)nx * ny;
    double aM = 0.0, aEs = 0.0, aEm = 0.0, aS2 = 0.0;
    for (int tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int x0 = (tile % tiles_x) * kNaTx;
        const int y0 = (tile / tiles_x) * kNaTy;
        __syncthreads();  // the previous tile's reads of ps and rh are done
        for (int cell = tid; cell < kNaLx * kNaLy; cell += kNaThreads) {
            const int cx = cell % kNaLx, cy = cell / kNaLx;
            const int gx = na_wrap(x0 - 2 + cx, nx), gy = na_wrap(y0 - 2 + cy, ny);
            const int64_t s = (int64_t)gy * nx + gx;
            C v[9];
#pragma unroll
            for (int i = 0; i < 9; ++i)
                v[i] = na_ld<S, C>(f + i * N + s, i == 0 ? k.o0 : (i < 5 ? k.o1 : k.o2));
            const C rho = ((v[0] + (v[1] + v[3])) + (v[2] + v[4])) + ((v[5] + v[7]) + (v[6] + v[8]));
            ps[cy][cx] = k.sqrt_rho0 * ((C)1 - na_exp(-rho * k.inv_rho0));
            if (cx >= 2 && cx < kNaTx + 2 && cy >= 2 && cy < kNaTy + 2) rh[cy - 2][cx - 2] = rho;
        }
        __syncthreads();
        if (x0 + tx < nx && y0 + ty < ny) {
            // psi at (x + dx, y + dy): row ty + 2 + dy, column tx + 2 + dx.
            auto q = [&](int dx, int dy) { return ps[ty + 2 + dy][tx + 2 + dx]; };
            const C p = q(0, 0);
            const C S1 = (q(1, 0) + q(-1, 0)) + (q(0, 1) + q(0, -1));
            const C S2 = (q(1, 1) + q(-1, -1)) + (q(-1, 1) + q(1, -1));
            const C S4 = (q(2, 0) + q(-2, 0)) + (q(0, 2) + q(0, -2));
            const C S5 = ((q(2, 1) + q(-2, -1)) + (q(2, -1) + q(-2, 1))) +
                         ((q(1, 2) + q(-1, -2)) + (q(-1, 2) + q(1, -2)));
            const C S8 = (q(2, 2) + q(-2, -2)) + (q(-2, 2) + q(2, -2));
            const C es = (C)0.5 * p * (k.KE0 * p + k.K1 * S1 + k.K2 * S2);
            const C em = (C)0.5 * p * (k.K4 * S4 + k.K5 * S5 + k.K8 * S8);
            aM += (double)rh[ty][tx];
            aEs += (double)es;
            aEm += (double)em;
            aS2 += (double)p * (double)p;
        }
    }
    double v[4] = {aM, aEs, aEm, aS2};
    const int lane = tid & 63, wid = tid >> 6;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        v[q] = na_wave_sum(v[q]);
        if (lane == 0) red[q][wid] = v[q];
    }
    __syncthreads();
    if (tid < 4) {
        double s = 0.0;
        for (int w = 0; w < kNaThreads / 64; ++w) s += red[tid][w];
        part[(int64_t)blockIdx.x * 4 + tid] = s;
    }
}

// One workgroup: fixed-order sums of the partials into the row
// {t, M, E_s, E_m, sum psi^2, E_bulk}.
__global__ void __launch_bounds__(256)
k_na_final(const double* __restrict__ part, int blocks, double t, double half_A1,
           double* __restrict__ row)
{
    __shared__ double sm[4][256];
    const int tid = threadIdx.x;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        double s = 0.0;
        for (int b = tid; b < blocks; b += 256) s += part[(int64_t)b * 4 + q];
        sm[q][tid] = s;
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w)
#pragma unroll
            for (int q = 0; q < 4; ++q) sm[q][tid] += sm[q][tid + w];
        __syncthreads();
    }
    if (tid == 0) {
        row[0] = t;
        row[1] = sm[0][0];
        row[2] = sm[1][0];
        row[3] = sm[2][0];
        row[4] = sm[3][0];
        row[5] = half_A1 * sm[3][0];
    }
}

template <typename S, typename C>
hipError_t na_run(const void* state, int nx, int ny, const Coef& c, const float* cf, double t,
                  double half_A1, double* out, hipStream_t s)
{
    double* sp = nullptr;
    hipError_t e = scratch_ptr(&sp);
    if (e != hipSuccess) return e;
    NaCoef<S, C> k;
    if constexpr (sizeof(C) == 8) {
        k = NaCoef<S, C>{c.KE0, c.K1, c.K2, c.K4, c.K5, c.K8, c.sqrt_rho0, c.inv_rho0, 0.0, 0.0, 0.0};
    } else {
        // The single-precision coefficients exactly as the step launchers pass
        // them: K1, K2, K4, K5, K8, KE0, tau, omega, sqrt_rho0, inv_rho0, rho_ref.
        k.K1 = cf[0];
        k.K2 = cf[1];
        k.K4 = cf[2];
        k.K5 = cf[3];
        k.K8 = cf[4];
        k.KE0 = cf[5];
        k.sqrt_rho0 = cf[8];
        k.inv_rho0 = cf[9];
        {
            // The offsets of the step kernels (dev_axis_offset).
            const float a = sizeof(S) == 2 ? dev_axis_offset(cf[10]) : 0.0f;
            k.o1 = a;
            k.o0 = 4.0f * a;
            k.o2 = 0.25f * a;
        }
    }
    const int tiles = ((nx + kNaTx - 1) / kNaTx) * ((ny + kNaTy - 1) / kNaTy);
    const int blocks = tiles < kNaBlocks ? tiles : kNaBlocks;
    if (blocks * 4 + 6 > kNaScratchDoubles) return hipErrorInvalidValue;  // never: blocks <= kNaBlocks
    hipLaunchKernelGGL((k_na_energy<S, C>), dim3(blocks), dim3(kNaThreads), 0, s,
                       static_cast<const S*>(state), nx, ny, k, sp);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    double* row = sp + kNaBlocks * 4;
    hipLaunchKernelGGL(k_na_final, dim3(1), dim3(256), 0, s, sp, blocks, t, half_A1, row);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(out, row, 6 * sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess)
        return e;
    return hipStreamSynchronize(s);
}

}  // namespace

hipError_t noalloc_energy(int storage, const void* state, int nx, int ny, const Coef& c, double t,
                          double half_A1, double* out, hipStream_t s)
{
    float cf[13];
    coef_to_f32(c, cf);
    switch (storage) {
    case ST_F64: return na_run<double, double>(state, nx, ny, c, cf, t, half_A1, out, s);
    case ST_F32: return na_run<float, float>(state, nx, ny, c, cf, t, half_A1, out, s);
    case ST_F16DEV: return na_run<_Float16, float>(state, nx, ny, c, cf, t, half_A1, out, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace lbk
