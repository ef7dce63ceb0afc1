// Internal interface between the C ABI (lb_api.hip) and the HIP kernels
// (lb_kernels.hip).  Not installed; the public interface is include/lb.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lbk {

// Population storage codes (same values as enum lb_storage).
enum Storage { ST_F64 = 0, ST_F32 = 1, ST_F16DEV = 2 };

// Work done by one launch of the step kernel.
enum Mode {
    MODE_STEP = 0,         // stream + collide + store
    MODE_STEP_ENERGY = 1,  // the same, plus the energy/mass block partials
    MODE_ENERGY = 2,       // energy/mass block partials only, no store
    MODE_STEP_TAPE = 3     // stream + collide + store, plus (rho, jx, jy, psi)
                           // of every site's pre-collision state into a dense
                           // [4][ny][nx] array of the arithmetic type, passed
                           // in place of the partials (F64 and F32 only)
};

// Lattice geometry and launch shape.  Populations live in two buffers of
// 9 planes each; plane i holds population i as ny rows of `pitch` elements
// (x fastest, pitch a multiple of 64 elements), planes `plane` elements apart.
struct Geom {
    int32_t nx, ny;
    int32_t pitch;    // elements per row; ny * pitch < 2^31
    int64_t plane;    // elements per population plane
    int32_t tile_x;   // columns per workgroup (= threads per workgroup)
    int32_t tile_y;   // rows per workgroup
    int32_t tiles_x;  // column strips
    int32_t blocks;   // workgroups of the step kernel
    int32_t rows_per_iter;  // rows each workgroup updates per pipeline stage (1 or 2)
};

// Physical coefficients, in double; the launchers convert them to the
// arithmetic precision of the storage.
// Half storage: the populations are kept as deviations f_i - w_i rho' from
// offsets built on one single-precision value a = rho'/9 (the axis offset):
// a is rho_ref/9 rounded to 20 significant bits, so that the rest offset
// 4a, the diagonal offset a/4 and the sum of all nine offsets, 9a, are
// exact.  The encoder subtracts that sum from the density; were it rounded,
// every site would gain the same rounding error at every step, a drift of
// the total mass linear in time.
__host__ __device__ inline float dev_axis_offset(float rho_ref)
{
    float v = rho_ref * (1.0f / 9.0f);
    uint32_t u;
    __builtin_memcpy(&u, &v, sizeof u);
    u = (u + 8u) & ~15u;  // nearest value with the low 4 significand bits clear
    __builtin_memcpy(&v, &u, sizeof v);
    return v;
}

struct Coef {
    double K1, K2, K4, K5, K8;  // link coupling of each |c|^2 class (Table 1)
    double KE0;                 // rest coupling of E_s: G1 w_0 + G2 p_s0
    double tau, omega;          // BGK relaxation time and 1/tau
    double sqrt_rho0, inv_rho0; // psi = sqrt(rho0) (1 - exp(-rho/rho0))
    double rho_ref;             // deviation reference of ST_F16DEV
    uint32_t step;              // time step of the launch
};

// One lattice of a batch, as the batched kernels read it (device memory).
struct BatchLattice {
    Geom geom;
    Geom geom2;          // two-step geometry (used when the batch runs two steps per launch)
    Coef coef;
    void* buf[2];        // population buffers; the step reads buf[parity]
    double* trace;       // this lattice's trace rows
    double half_A1;      // (G1 + G2) / 2
    int32_t tile_begin;  // first logical tile of this lattice in the batch
    int32_t tile_begin2; // first logical tile of this lattice in the two-step tile list
    float coef_f[13];    // coef converted to single precision (coef_to_f32), so the
                         // single-precision kernels read it without converting
    int32_t pad;
};

// coef in single precision, exactly as the single-lattice launchers pass it:
// K1, K2, K4, K5, K8, KE0, tau, omega, sqrt_rho0, inv_rho0, rho_ref, 2 K4, 2 K8.
void coef_to_f32(const Coef& c, float out[13]);

// Bytes of one stored population value.
inline int storage_bytes(int storage)
{
    return storage == ST_F64 ? 8 : storage == ST_F32 ? 4 : 2;
}

hipError_t launch_step(int storage, int mode, const void* src, void* dst,
                       const Geom& g, const Coef& c, double* partials,
                       hipStream_t s);
// Two plain steps in one launch (ST_F32 and ST_F16DEV storage).  g is the two-step
// geometry: tile_x lanes produce tile_x - 6 output columns, tiles_x =
// ceil(nx / (tile_x - 6)), blocks = tiles_x * ceil(ny / tile_y).
hipError_t launch_step2(int storage, const void* src, void* dst, const Geom& g, const Coef& c,
                        hipStream_t s);
// Two plain steps of every lattice of a batch in one launch: tiles logical
// tiles of tile_x lanes, tile_lattice maps each to its lattice, whose geom2
// gives the tile's place; the launch reads buf[parity] and writes
// buf[parity ^ 1] of every lattice.
hipError_t launch_step2_batch(int storage, int tile_x, const BatchLattice* desc,
                              const int32_t* tile_lattice, int tiles, int parity, uint32_t step,
                              hipStream_t s);
// Workgroups of tile_x lanes of the two-step kernel (ST_F32 or ST_F16DEV)
// resident on the current device at once: the runtime's occupancy for the
// kernel's registers and LDS, per compute unit, times the compute units.
// -1 when no device can be asked.
int step2_resident(int storage, int tile_x);
hipError_t launch_final(const double* partials, int blocks, double t,
                        double half_A1, double* out_row, hipStream_t s);
hipError_t launch_step_batch(int storage, int mode, int tile_x, int rows_per_iter, int min_tile_y,
                             const BatchLattice* desc, const int32_t* tile_lattice, int tiles,
                             int parity, uint32_t step, double* partials, hipStream_t s);
hipError_t launch_final_batch(const BatchLattice* desc, int count, const double* partials,
                              double t, int64_t row, hipStream_t s);
hipError_t launch_moments(int storage, const void* src, const Geom& g,
                          const Coef& c, double* rho, double* ux, double* uy,
                          hipStream_t s);
hipError_t launch_init(int storage, const double* rho, const double* ux,
                       const double* uy, void* dst, const Geom& g,
                       const Coef& c, hipStream_t s);
hipError_t launch_get_state(int storage, const void* src, void* dense,
                            const Geom& g, hipStream_t s);
hipError_t launch_set_state(int storage, const void* dense, void* dst,
                            const Geom& g, hipStream_t s);

// Section V observables {t, M, E_s, E_m, sum psi^2, E_bulk} of a dense
// [9][ny][nx] pre-collision population array of the given storage (device
// memory) into out (host, 6 doubles), with every intermediate in the
// library's static device scratch (lb_noalloc.hip): no allocation, and the
// stream is synchronised before returning.
hipError_t noalloc_energy(int storage, const void* state, int nx, int ny, const Coef& c, double t,
                          double half_A1, double* out, hipStream_t s);

// Adjoint kernels (lb_adjoint.hip).  Arithmetic is double when f64 != 0,
// float otherwise; arrays are dense [component][ny][nx] of that type.
struct AdjParams {
    int32_t nx, ny;
    int32_t f64;
    double G1, G2, tau, sqrt_rho0, inv_rho0;
};

// Workgroups of every per-site adjoint kernel (one thread per site).
int adj_blocks(int64_t sites);
// tape[4][ny][nx] = (rho, jx, jy, psi) of the state held in a pitched
// population buffer of the given storage (ST_F64 or ST_F32).
hipError_t adj_tape(int storage, const void* buf, const Geom& g, const AdjParams& p, void* tape,
                    hipStream_t s);
// One adjoint step: (lam_next, g_next) at t+1 -> (lam, g) at t; gF[2][ny][nx]
// is scratch; part[adj_blocks][2] accumulates dL/dG1, dL/dG2.
hipError_t adj_step(const AdjParams& p, const void* lam_next, const void* g_next, const void* tape,
                    void* lam, void* g, void* gF, double* part, hipStream_t s);
// Interface measure of a tape entry: dir[2][ny][nx], part[adj_blocks] sums.
hipError_t adj_area(const AdjParams& p, const void* tape, double eps, void* dir, double* part,
                    hipStream_t s);
// Adjoint at T of L = (E - E*)^2 + beta A; part[adj_blocks][2] receives the
// workgroup sums of dE/dG1, dE/dG2.
hipError_t adj_seed(const AdjParams& p, const void* tape, const void* dir, double two_dE, double beta,
                    void* lam, void* g, double* part, hipStream_t s);
// out[ny][nx] (double) = sum_i w_i (lam_i + g).
hipError_t adj_rho_grad(const AdjParams& p, const void* lam, const void* g, double* out, hipStream_t s);
// out[v] = sum_b part[b * nv + v] for v < nv, fixed order.
hipError_t adj_reduce(const double* part, int blocks, int nv, double* out, hipStream_t s);
hipError_t adj_zero(double* p, int64_t n, hipStream_t s);

// Structure factor (lb_structure.hip) of an L x L density field, L <= kSkMaxL.
constexpr int kSkMaxL = 2048;
struct SkPlan {
    int32_t L;
    int32_t logL;        // log2 L if L is a power of two, else 0 (direct DFT)
    int32_t nshell;      // shells 0 .. nshell-1
    int32_t sum_blocks;  // workgroups of the mean reduction
    double2* tw;         // L twiddles exp(-2 pi i k / L)
    double* part;        // sum_blocks partial sums
    double* mean;        // 1
    double2* z;          // L*L: row transforms, [y][l]
    double2* zt;         // L*L: their transpose, [l][y]
    double* spec_t;      // L*L: S at (l, m), stored [l][m]
    const int32_t* idx;  // L*L: indices into spec_t, grouped by shell
    const int32_t* off;  // nshell + 1: shell n is idx[off[n] .. off[n+1])
    double* shell;       // nshell shell averages
    double* kbar;        // 2: {kbar, sum_n S_n}
};
// Runs every pass on rho (device, L*L doubles); spectrum (device, [m][l])
// may be NULL.
hipError_t sk_compute(const SkPlan& p, const double* rho, double* spectrum, hipStream_t s);
// Fills p.tw (once per plan).
hipError_t sk_twiddles(const SkPlan& p, hipStream_t s);

}  // namespace lbk
