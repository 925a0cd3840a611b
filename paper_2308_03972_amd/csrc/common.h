// Internal declarations shared by the HIP translation units of liblbmletkf.
// Device-side lattice constants, wave helpers and the kernel launchers that
// the C-ABI layer (api.hip) calls.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace lbmletkf {

// D2Q9 (Sec. 2): velocity order 0:(0,0) 1:(1,0) 2:(-1,0) 3:(0,1) 4:(0,-1)
// 5:(1,1) 6:(-1,-1) 7:(1,-1) 8:(-1,1); weights 4/9, 1/9 (axis), 1/36 (diagonal).
__host__ __device__ constexpr int cx_of(int a) {
    return (a == 1 || a == 5 || a == 7) ? 1 : (a == 2 || a == 6 || a == 8) ? -1 : 0;
}
__host__ __device__ constexpr int cy_of(int a) {
    return (a == 3 || a == 5 || a == 8) ? 1 : (a == 4 || a == 6 || a == 7) ? -1 : 0;
}
__host__ __device__ constexpr double w_of(int a) {
    return a == 0 ? 4.0 / 9.0 : (a <= 4 ? 1.0 / 9.0 : 1.0 / 36.0);
}

constexpr int kWave = 64;

// Population storage layout: [node][a][member], node = y * nx + x, members
// fastest, so the M values of one population of one node are contiguous and a
// wavefront of 64 members reads or writes 512 contiguous bytes (FP64).
__host__ __device__ __forceinline__ size_t slot(size_t node, int a, int m, int members) {
    return (node * 9 + (size_t)a) * (size_t)members + (size_t)m;
}
__host__ __device__ __forceinline__ int wrap1(int i, int n) {
    return i < 0 ? i + n : (i >= n ? i - n : i);
}
// Under pull streaming the canonical f_a of node (x, y) is held by the slot
// of node (x - c_ax, y - c_ay).
__host__ __device__ __forceinline__ size_t src_node(int x, int y, int a, int nx, int ny) {
    return (size_t)wrap1(y - cy_of(a), ny) * nx + wrap1(x - cx_of(a), nx);
}
// The storage slots a thread of node (x, y), member m pulls from: the slot of
// population a at node (x - c_ax, y - c_ay).  Three row pointers (64-bit, one
// multiply each) and three column offsets within a row (32-bit: a lattice row
// holds nx * 9 * members < 2^31 slots, checked when a context is created), so
// that each of the nine sources costs a 32-bit add and a pointer add instead
// of a 64-bit multiply-add chain (60-130 fewer instructions per thread in the
// forecast and adjoint kernels).  The FP32 two-step forecast is issue-bound and
// gains from it; the FP64 kernels wait on memory and keep their time.
// xm, xp, ym, yp: the wrapped neighbours x - 1, x + 1, ...
template <typename P>
struct PullSlots {
    P* rows[3];       // row y - c_ay, indexed c_ay + 1
    uint32_t cols[3]; // column offset (x - c_ax) * 9 M + m, indexed c_ax + 1
    uint32_t members;
    __device__ __forceinline__ PullSlots(P* base, int x, int xm, int xp, int y, int ym, int yp,
                                         int nx, int members_, int m)
        : members((uint32_t)members_) {
        const size_t row = (size_t)nx * 9 * members_;
        rows[0] = base + (size_t)yp * row;
        rows[1] = base + (size_t)y * row;
        rows[2] = base + (size_t)ym * row;
        const uint32_t node = 9u * members;
        cols[0] = (uint32_t)xp * node + (uint32_t)m;
        cols[1] = (uint32_t)x * node + (uint32_t)m;
        cols[2] = (uint32_t)xm * node + (uint32_t)m;
    }
    // a: a compile-time constant after unrolling
    __device__ __forceinline__ P* at(int a) const {
        return rows[cy_of(a) + 1] + (cols[cx_of(a) + 1] + (uint32_t)a * members);
    }
};

// Node-member launches: blocks of (members, nodes_per_block) threads.
inline int nodes_per_block(int members) { return members >= 256 ? 1 : 256 / members; }

// Population storage: FP64 values f, or FP32 deviations f - w from the lattice
// weights (the precision form).  Arithmetic is FP64 in both cases; only the
// bytes kept in HBM differ.
enum Storage { kStoreF64 = 0, kStoreF32Dev = 1 };

template <typename T>
struct PopIO;

template <>
struct PopIO<double> {
    __device__ static double load(const double* p, int) { return *p; }
    __device__ static double load_nt(const double* p, int) { return __builtin_nontemporal_load(p); }
    __device__ static void store(double* p, int, double v) { *p = v; }
    __device__ static void store_nt(double* p, int, double v) { __builtin_nontemporal_store(v, p); }
    // the value a store followed by a load gives back
    __device__ static double round(double v, int) { return v; }
};

template <>
struct PopIO<float> {
    __device__ static double load(const float* p, int a) { return w_of(a) + (double)*p; }
    __device__ static double load_nt(const float* p, int a) {
        return w_of(a) + (double)__builtin_nontemporal_load(p);
    }
    __device__ static void store(float* p, int a, double v) { *p = (float)(v - w_of(a)); }
    __device__ static void store_nt(float* p, int a, double v) {
        __builtin_nontemporal_store((float)(v - w_of(a)), p);
    }
    __device__ static double round(double v, int a) { return w_of(a) + (double)(float)(v - w_of(a)); }
};

inline size_t state_elem_bytes(int storage) { return storage == kStoreF32Dev ? 4 : 8; }

// Stage identifiers for per-launch timing.
enum Stage { kStageCollide = 0, kStageObserve = 1, kStageStats = 2, kStageAnalysis = 3,
             kStageDiag = 4, kStageAdjoint = 5, kStageMisfit = 6, kNumStages = 7 };

struct LbmDims {
    int nx, ny, members;
};

// ---- lattice-Boltzmann kernels (lbm_kernels.hip) -------------------------
// One fused pull-stream + BGK-Smagorinsky collide step, fin -> fout (storage layout).
// `storage` selects the element type of every state buffer (Storage).
hipError_t launch_stream_collide(const void* fin, void* fout, const double* force, LbmDims d,
                                 double tau0, double cs, double mu, int storage, hipStream_t s);
// Two such steps in one launch (spatial tiles with a recomputed one-node ring,
// the intermediate state in LDS); needs two_step_supported(d).  Same
// arithmetic and rounding as two launches of launch_stream_collide; with fmid
// != NULL the intermediate state is written there too (the first launch's
// output).
bool two_step_supported(LbmDims d, int storage);
hipError_t launch_stream_collide2(const void* fin, void* fout, const double* force, LbmDims d,
                                  double tau0, double cs, double mu, int storage, hipStream_t s,
                                  void* fmid = nullptr);
// One problem of a batched forecast step: its state buffers (storage layout),
// force, sizes, relaxation parameters and its first tile in the batch.
struct LbmTask {
    const void* fin;
    void* fout;
    const double* force;
    int nx, ny, members;  // members divides 256
    int tile_nodes;       // nodes per tile (a multiple of 256 / members)
    int tile0;            // first tile of this problem in the concatenated list
    int block0;           // first block of this problem in a batched two-step launch
    double tau0, smag, mu;
};
// All problems' steps in one persistent launch of `blocks` blocks over `ntiles` tiles.
hipError_t launch_stream_collide_batch(const LbmTask* d_tasks, int ntasks, int ntiles, int blocks,
                                       int storage, hipStream_t s);
// Blocks of one problem's two-step launch in a batch (tiles x member groups of
// 16, or of 32 for FP32 storage with 32 | members; needs 16 | members), and two
// steps of all problems in one launch over the concatenated block list
// (nblocks = sum of two_step_blocks); the same arithmetic and rounding as the
// single-problem two-step launch.
int two_step_blocks(LbmDims d, int storage);
hipError_t launch_stream_collide2_batch(const LbmTask* d_tasks, int ntasks, int nblocks,
                                        int storage, hipStream_t s);
hipError_t launch_import(const double* canon, void* f, LbmDims d, int storage, hipStream_t s);
hipError_t launch_export(const void* f, double* canon, LbmDims d, int storage, hipStream_t s);
hipError_t launch_init_equilibrium(const double* rho, const double* uv, void* f, LbmDims d,
                                   int storage, hipStream_t s);
hipError_t launch_moments(const void* f, double* out, LbmDims d, int storage, hipStream_t s);

// ---- observation, statistics, analysis, diagnostics (letkf_kernels.hip) ---
hipError_t launch_observe(const void* f, const int* pts, int npts, int nvar, double* yf,
                          LbmDims d, int storage, hipStream_t s);
// y_bar, dY, d = y^o - y_bar and (K != NULL) the Gram matrix K = dY dY^T on the
// matrix cores: FP64 MFMA, or FP32 MFMA for the precision form's storage.
hipError_t launch_obs_stats(const double* yf, const double* yo, int nobs, int members,
                            double* ybar, double* dY, double* dvec, double* K, int storage,
                            hipStream_t s);
hipError_t launch_local_table(const int* pts, int npts, double d_cut, int lmax, int nx, int ny,
                              int* loc_pt, double* loc_g, int* overflow, hipStream_t s);

struct AnalysisParams {
    void* f;              // storage layout [M][9][ny][nx], updated in place
    int storage;          // Storage of f
    int nx, ny, members;
    const double* dY;     // [nobs][M] forecast observation perturbations
    const double* K;      // [nobs][nobs] = dY dY^T (observation route)
    const double* dvec;   // [nobs] innovation y^o - y_bar
    const int* loc_pt;    // [nx*ny][lmax] local observation points, -1 = empty
    const double* loc_g;  // [nx*ny][lmax] Gaspari-Cohn weights
    int lmax, nvar, nobs;
    double rinv[3];       // 1 / sigma^2 per variable
    double a;             // (M - 1) / beta
    double sqrt_beta;
    int max_sweeps;       // Jacobi sweep cap of the eigensolvers
    int mfma_transform;   // FP32 storage: B = dX Z^T and the transform on BF16 matrix cores
    int* eig_fail;        // count of nodes whose eigensolver hit the sweep cap
    // cycle diagnostics folded into the analysis (NULL: none): per node the five
    // diagnostic fields (err2, spread2, non-finite, rho min, rho max) of the
    // forecast at diag_node[node * 5] and of the analysis at
    // diag_node[(plane + node) * 5]; truth_uv [2][ny][nx] or NULL (err2 = 0)
    const double* truth_uv;
    double* diag_node;
};
// Fields of one diagnostics record.
constexpr int kDiagFieldCount = 5;
// Reduce the per-node records of the forecast and the analysis (in fixed
// order) into two diagnostics outputs; `partial` holds
// 2 * diag_fold_blocks(plane) * kDiagFieldCount doubles.
int diag_fold_blocks(int plane);
hipError_t launch_diag_nodes_final(const double* diag_node, int plane, double* partial,
                                   double* out_forecast, double* out_analysis, hipStream_t s);
// Ensemble route (M x M eigenproblem of size n >= M), every node.
hipError_t launch_analysis_ens(const AnalysisParams& p, int n, hipStream_t s);
int ens_size_for(int n);              // instantiated size >= n, or 0
int ens_lds_bytes(int n, int nz);
int ens_segments(int n);              // nodes per wavefront of the ensemble route
// Batched ensemble route: wavefront w handles waves[w] = (problem, first node of
// its ens_segments(n) consecutive nodes of that problem); nz_max
// is the largest nvar * lmax among the problems.
hipError_t launch_analysis_ens_batch(const AnalysisParams* d_params, const int2* d_waves,
                                     int nwaves, int n, int nz_max, int storage, hipStream_t s);
// Observation route (l x l dual, size n >= l) for the `count` nodes listed in
// `nodes`; gbuf holds obs_gbuf_doubles(n, count) doubles (per-node G and h
// passed from the eigen kernel to the apply kernel).
hipError_t launch_analysis_obs(const AnalysisParams& p, const int* nodes, int count, int n,
                               double* gbuf, hipStream_t s);
int obs_size_for(int n);              // instantiated size >= n, or 0
int obs_lds_bytes(int n);             // the larger of the two kernels' LDS
size_t obs_gbuf_doubles(int n, int count);
int obs_segments(int n);              // nodes per wavefront of the eigen kernel
// Batched observation route for one eigenproblem size n over many problems:
// eigen wavefront w handles eig_waves[w] = (problem, first item, end of that
// problem's items, -); apply wavefront w handles apply_waves[w] = (problem, item);
// items index the shared node list and G buffer; d_params[problem] is that
// problem's AnalysisParams.
hipError_t launch_analysis_obs_batch(const AnalysisParams* d_params, const int4* d_eig_waves,
                                     int n_eig, const int2* d_apply_waves, int n_apply,
                                     const int* d_nodes, int n, double* gbuf, int storage,
                                     bool mfma_transform, hipStream_t s);
// The same with persistent launches that take the wave lists' entries from
// queues: counters[0..7] (eigen) and counters[8..15] (apply), zero on entry.
hipError_t launch_analysis_obs_batch_queue(const AnalysisParams* d_params, const int4* d_eig_waves,
                                           int n_eig, const int2* d_apply_waves, int n_apply,
                                           const int* d_nodes, int n, double* gbuf, int storage,
                                           bool mfma_transform, int* counters, hipStream_t s);
// Zero n ints with a kernel (capturable in a graph, unlike hipMemsetAsync).
hipError_t launch_zero_ints(int* v, int n, hipStream_t s);
int diag_blocks_for(int plane);
// Bytes of diag_partial_kernel's per-block records for a grid of `plane` nodes.
size_t diag_partial_bytes(int plane);
// The static device scratch (kStaticScratchBytes) of the allocation-free
// entry point: its device address on the current device, resolved once per
// device (hipGetSymbolAddress) and kept.
constexpr size_t kStaticScratchBytes = size_t(4) << 20;
hipError_t static_scratch(void** addr);

hipError_t launch_diag(const void* f, const double* truth_uv, LbmDims d, int storage,
                       double* partial, int nblocks, double* out, hipStream_t s);
hipError_t launch_synth_obs(const double* y, const double* eps, const double* sigma, double* yo,
                            int n, hipStream_t s);

// ---- energy spectrum (spectrum.hip) ----------------------------------------
// Member-mean shell spectrum E[0..kmax] of the velocity of an n x n ensemble;
// `scratch` holds spectrum_scratch_bytes(n, members) bytes (256-byte aligned).
size_t spectrum_scratch_bytes(int n, int members);
hipError_t launch_energy_spectrum(const void* f, int n, int members, int storage, int kmax,
                                  void* scratch, double* E, hipStream_t s);

// ---- differentiation form (adjoint.hip) -----------------------------------
// One reverse step: lam_out = adjoint of the step taken from fstate (storage
// layout) applied to lam_in; adjoint states are FP64 in the canonical
// node-major layout [node][a][member] (unshifted); each block adds
// its share of d(lam_in . step)/dK, K = 18 sqrt(2) C_s^2, to k_partial[block].
int adjoint_partials(LbmDims d);
hipError_t launch_adjoint_step(const void* fstate, const double* lam_in, double* lam_out,
                               const double* force, LbmDims d, double tau0, double cs, double mu,
                               int storage, double* k_partial, hipStream_t s);
// Misfit terms at one observation time: jbuf[m * npts + k] += sum_var (H - y^o)^2
// (jbuf may be NULL); if lam is not NULL, lam += dJ/df at the observation
// nodes (the points must be distinct).
hipError_t launch_misfit(const void* f, const int* pts, int npts, int nvar, const double* yo,
                         double* lam, double* jbuf, LbmDims d, int storage, hipStream_t s);
// Adjoint state [node][a][member] -> canonical [member][a][y][x].
hipError_t launch_lam_to_canonical(const double* lam, double* out, LbmDims d, hipStream_t s);
hipError_t launch_sum(const double* v, size_t n, double scale, double* out, hipStream_t s);
hipError_t launch_fill(double* v, size_t n, double value, hipStream_t s);

}  // namespace lbmletkf
