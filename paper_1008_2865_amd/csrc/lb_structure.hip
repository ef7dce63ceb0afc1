// Structure factor of the density field (the Fourier analysis of section
// IV): S(k) = (1/N) |sum_x (rho(x) - mean rho) e^{i k.x}|^2 on the modes
// k = (2 pi / L)(l, m) of an L x L lattice, its average over the circular
// shells (n - 1/2) <= |k| L / 2 pi < n + 1/2 and the first moment
// kbar = sum_n n S_n / sum_n S_n (eq. (rad), k in units of 2 pi / L).
//
// The 2-D transform is a row pass, a transpose and a column pass; each pass
// transforms one line per workgroup in LDS, in double precision: a radix-2
// decimation-in-time FFT when L is a power of two, the direct sum over x
// otherwise, with twiddles from a table computed once (sincospi).  The
// transposes are 32 x 32 LDS tiles, so every global access is coalesced.  The sign of the exponent does not matter for |.|^2 of a
// real field (S(k) = S(-k)); the passes use e^{-i k.x}.  Shell sums run
// over a host-built list of the modes of each shell in increasing index
// order, one workgroup per shell: every sum has a fixed order, so results
// are bit-reproducible.
#include "lb_internal.h"

#include <hip/hip_runtime.h>

namespace lbk {
namespace {

constexpr int kThreads = 256;
constexpr int kTile = 32;

// Fixed-order workgroup sum (256 threads); the result is valid in thread 0.
__device__ __forceinline__ double block_reduce(double v, double* sm)
{
    const int tid = threadIdx.x;
    sm[tid] = v;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (tid < w) sm[tid] += sm[tid + w];
        __syncthreads();
    }
    return sm[0];
}

// part[b] = sum of rho[s] over s = b*256 + tid + k*gridDim*256.
__global__ void __launch_bounds__(kThreads)
k_sk_sum(const double* __restrict__ rho, int64_t N, double* __restrict__ part)
{
    __shared__ double sm[kThreads];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * kThreads)
        s += rho[i];
    const double t = block_reduce(s, sm);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// mean[0] = (sum of the partials) / N.
__global__ void __launch_bounds__(kThreads)
k_sk_mean(const double* __restrict__ part, int blocks, int64_t N, double* __restrict__ mean)
{
    __shared__ double sm[kThreads];
    double s = 0.0;
    for (int b = threadIdx.x; b < blocks; b += kThreads) s += part[b];
    const double t = block_reduce(s, sm);
    if (threadIdx.x == 0) mean[0] = t / (double)N;
}

// tw[k] = exp(-2 pi i k / L), k < L (once per context).
__global__ void __launch_bounds__(kThreads) k_sk_twiddles(int L, double2* __restrict__ tw)
{
    const int k = blockIdx.x * kThreads + threadIdx.x;
    if (k >= L) return;
    double s, c;
    sincospi(-2.0 * (double)k / (double)L, &s, &c);
    tw[k] = make_double2(c, s);
}

// One line of length L per workgroup.  kRows: the line is row `line` of
// rho minus its mean (real); otherwise row `line` of the complex array zin.
// kSpec: write |X_k|^2 * invN to spec[line * L + k]; otherwise X_k to
// zout[line * L + k].  Dynamic LDS: 2 L doubles (FFT) or 4 L (direct sum,
// which also keeps the twiddles in LDS).
template <bool kPow2, bool kRows, bool kSpec>
__global__ void __launch_bounds__(kThreads)
k_sk_line(const double* __restrict__ rho, const double* __restrict__ mean,
          const double2* __restrict__ zin, const double2* __restrict__ tw, int L, int logL,
          double invN, double2* __restrict__ zout, double* __restrict__ spec)
{
    extern __shared__ double lds[];
    double* re = lds;
    double* im = lds + L;
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * L;
    const double mu = kRows ? mean[0] : 0.0;
    for (int x = tid; x < L; x += kThreads) {
        double vr, vi;
        if (kRows) {
            vr = rho[base + x] - mu;
            vi = 0.0;
        } else {
            const double2 z = zin[base + x];
            vr = z.x;
            vi = z.y;
        }
        // Bit-reversed order for the in-place radix-2 passes.
        const int d = kPow2 ? (int)(__brev((unsigned)x) >> (32 - logL)) : x;
        re[d] = vr;
        im[d] = vi;
    }

    auto emit = [&](int k, double xr, double xi) {
        if (kSpec)
            spec[base + k] = (xr * xr + xi * xi) * invN;
        else
            zout[base + k] = make_double2(xr, xi);
    };

    if (kPow2) {
        __syncthreads();
        for (int half = 1; half < L; half <<= 1) {
            const int step = L / (2 * half);
            for (int b = tid; b < L / 2; b += kThreads) {
                const int pos = b & (half - 1);
                const int i = ((b - pos) << 1) + pos;
                const int j = i + half;
                const double2 w = tw[pos * step];
                const double xr = re[j] * w.x - im[j] * w.y;
                const double xi = re[j] * w.y + im[j] * w.x;
                const double ar = re[i], ai = im[i];
                re[i] = ar + xr;
                im[i] = ai + xi;
                re[j] = ar - xr;
                im[j] = ai - xi;
            }
            __syncthreads();
        }
        for (int k = tid; k < L; k += kThreads) emit(k, re[k], im[k]);
    } else {
        double* twc = lds + 2 * L;
        double* tws = lds + 3 * L;
        for (int k = tid; k < L; k += kThreads) {
            const double2 w = tw[k];
            twc[k] = w.x;
            tws[k] = w.y;
        }
        __syncthreads();
        // X_k = sum_x v_x w^{(x k) mod L}.
        for (int k = tid; k < L; k += kThreads) {
            double sr = 0.0, si = 0.0;
            int t = 0;
            for (int x = 0; x < L; ++x) {
                const double wr = twc[t], wi = tws[t];
                sr += re[x] * wr - im[x] * wi;
                si += re[x] * wi + im[x] * wr;
                t += k;
                if (t >= L) t -= L;
            }
            emit(k, sr, si);
        }
    }
}

// out[c][r] = in[r][c] for an L x L array, through 32 x 32 LDS tiles.
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_sk_transpose(const T* __restrict__ in, int L, T* __restrict__ out)
{
    __shared__ T tile[kTile][kTile + 1];
    const int tx = threadIdx.x & (kTile - 1), ty = threadIdx.x / kTile;  // 32 x 8
    const int c0 = blockIdx.x * kTile, r0 = blockIdx.y * kTile;
    for (int r = ty; r < kTile; r += kThreads / kTile) {
        const int gr = r0 + r, gc = c0 + tx;
        if (gr < L && gc < L) tile[r][tx] = in[(int64_t)gr * L + gc];
    }
    __syncthreads();
    for (int c = ty; c < kTile; c += kThreads / kTile) {
        const int gc = c0 + c, gr = r0 + tx;
        if (gr < L && gc < L) out[(int64_t)gc * L + gr] = tile[tx][c];
    }
}

// Shell n (one workgroup each): average of spec over its modes, listed in
// idx[off[n] .. off[n+1]).
__global__ void __launch_bounds__(kThreads)
k_sk_shell(const double* __restrict__ spec, const int32_t* __restrict__ idx,
           const int32_t* __restrict__ off, double* __restrict__ shell)
{
    __shared__ double sm[kThreads];
    const int n = blockIdx.x;
    const int a = off[n], b = off[n + 1];
    double s = 0.0;
    int j = a + threadIdx.x;
    // Eight independent gathers in flight per thread, then the tail.
    for (; j + 7 * kThreads < b; j += 8 * kThreads) {
        double v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = spec[idx[j + q * kThreads]];
        s += ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
    }
    for (; j < b; j += kThreads) s += spec[idx[j]];
    const double t = block_reduce(s, sm);
    if (threadIdx.x == 0) shell[n] = b > a ? t / (double)(b - a) : 0.0;
}

// out = {kbar, sum_n S_n}: kbar = sum_n n S_n / sum_n S_n.
__global__ void __launch_bounds__(kThreads)
k_sk_kbar(const double* __restrict__ shell, int nsh, double* __restrict__ out)
{
    __shared__ double sm[kThreads];
    double num = 0.0, den = 0.0;
    for (int n = threadIdx.x; n < nsh; n += kThreads) {
        num += (double)n * shell[n];
        den += shell[n];
    }
    const double tn = block_reduce(num, sm);
    __syncthreads();
    const double td = block_reduce(den, sm);
    if (threadIdx.x == 0) {
        out[0] = tn / td;
        out[1] = td;
    }
}

template <bool kPow2>
hipError_t transform(const SkPlan& p, const double* rho, hipStream_t s)
{
    const int L = p.L;
    const double invN = 1.0 / ((double)L * (double)L);
    const size_t lds = (size_t)(kPow2 ? 2 : 4) * L * sizeof(double);
    const dim3 tgrid((L + kTile - 1) / kTile, (L + kTile - 1) / kTile);
    hipLaunchKernelGGL((k_sk_line<kPow2, true, false>), dim3(L), dim3(kThreads), lds, s, rho, p.mean,
                       nullptr, p.tw, L, p.logL, invN, p.z, nullptr);
    hipLaunchKernelGGL(k_sk_transpose<double2>, tgrid, dim3(kThreads), 0, s, p.z, L, p.zt);
    hipLaunchKernelGGL((k_sk_line<kPow2, false, true>), dim3(L), dim3(kThreads), lds, s, nullptr,
                       nullptr, p.zt, p.tw, L, p.logL, invN, nullptr, p.spec_t);
    return hipGetLastError();
}

}  // namespace

hipError_t sk_twiddles(const SkPlan& p, hipStream_t s)
{
    hipLaunchKernelGGL(k_sk_twiddles, dim3((p.L + kThreads - 1) / kThreads), dim3(kThreads), 0, s, p.L,
                       p.tw);
    return hipGetLastError();
}

hipError_t sk_compute(const SkPlan& p, const double* rho, double* spectrum, hipStream_t s)
{
    const int64_t N = (int64_t)p.L * p.L;
    hipLaunchKernelGGL(k_sk_sum, dim3(p.sum_blocks), dim3(kThreads), 0, s, rho, N, p.part);
    hipLaunchKernelGGL(k_sk_mean, dim3(1), dim3(kThreads), 0, s, p.part, p.sum_blocks, N, p.mean);
    hipError_t e = p.logL > 0 ? transform<true>(p, rho, s) : transform<false>(p, rho, s);
    if (e) return e;
    hipLaunchKernelGGL(k_sk_shell, dim3(p.nshell), dim3(kThreads), 0, s, p.spec_t, p.idx, p.off,
                       p.shell);
    hipLaunchKernelGGL(k_sk_kbar, dim3(1), dim3(kThreads), 0, s, p.shell, p.nshell, p.kbar);
    if (spectrum) {
        // spec_t is indexed [l][m]; the caller's layout is [m][l].
        const dim3 tgrid((p.L + kTile - 1) / kTile, (p.L + kTile - 1) / kTile);
        hipLaunchKernelGGL(k_sk_transpose<double>, tgrid, dim3(kThreads), 0, s, p.spec_t, p.L,
                           spectrum);
    }
    return hipGetLastError();
}

}  // namespace lbk
