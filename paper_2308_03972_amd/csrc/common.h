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

// Stage identifiers for per-launch timing.
enum Stage { kStageCollide = 0, kStageObserve = 1, kStageStats = 2, kStageAnalysis = 3,
             kStageDiag = 4, kNumStages = 5 };

struct LbmDims {
    int nx, ny, members;
};

// ---- lattice-Boltzmann kernels (lbm_kernels.hip) -------------------------
// One fused pull-stream + BGK-Smagorinsky collide step, fin -> fout (storage layout).
hipError_t launch_stream_collide(const double* fin, double* fout, const double* force,
                                 LbmDims d, double tau0, double cs, double mu, hipStream_t s);
hipError_t launch_import(const double* canon, double* f, LbmDims d, hipStream_t s);
hipError_t launch_export(const double* f, double* canon, LbmDims d, hipStream_t s);
hipError_t launch_init_equilibrium(const double* rho, const double* uv, double* f, LbmDims d,
                                   hipStream_t s);
hipError_t launch_moments(const double* f, double* out, LbmDims d, hipStream_t s);

// ---- observation, statistics, analysis, diagnostics (letkf_kernels.hip) ---
hipError_t launch_observe(const double* f, const int* pts, int npts, int nvar, double* yf,
                          LbmDims d, hipStream_t s);
hipError_t launch_obs_stats(const double* yf, const double* yo, int nobs, int members,
                            double* ybar, double* dY, double* dvec, double* K, hipStream_t s);
hipError_t launch_local_table(const int* pts, int npts, double d_cut, int lmax, int nx, int ny,
                              int* loc_pt, double* loc_g, int* overflow, hipStream_t s);

struct AnalysisParams {
    double* f;            // storage layout [M][9][ny][nx], updated in place
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
    int* eig_fail;        // count of nodes whose eigensolver hit the sweep cap
};
// Ensemble route (M x M eigenproblem of size n >= M), every node.
hipError_t launch_analysis_ens(const AnalysisParams& p, int n, hipStream_t s);
int ens_size_for(int n);              // instantiated size >= n, or 0
int ens_lds_bytes(int n, int nz);
// Observation route (l x l dual, size n >= l) for the `count` nodes listed in `nodes`.
hipError_t launch_analysis_obs(const AnalysisParams& p, const int* nodes, int count, int n,
                               hipStream_t s);
int obs_size_for(int n);              // instantiated size >= n, or 0
int obs_lds_bytes(int n);
int diag_blocks_for(int plane);

hipError_t launch_diag(const double* f, const double* truth_uv, LbmDims d, double* partial,
                       int nblocks, double* out, hipStream_t s);
hipError_t launch_synth_obs(const double* y, const double* eps, const double* sigma, double* yo,
                            int n, hipStream_t s);

}  // namespace lbmletkf
