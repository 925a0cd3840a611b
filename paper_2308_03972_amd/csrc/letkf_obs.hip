// Observation-route LETKF analysis (Sec. 3.2.1, Sec. 3.2.2): for a node with
// l local observations the M x M ensemble-space matrix
// (M-1)/beta I + Z^T Z (Z = R_loc^-1/2 dY, l x M) is eigendecomposed through
// its l x l dual Z Z^T: the dual's eigenpairs (lambda_i, u_i) give the
// eigenpairs ((M-1)/beta + lambda_i, Z^T u_i / sqrt(lambda_i)) and the
// eigenvalue (M-1)/beta on the orthogonal complement.  Hence
//   w_bar = Z^T U (a + Lambda)^-1 U^T d~,   a = (M-1)/beta,
//   dW    = sqrt(beta) I + Z^T U phi(Lambda) U^T Z,
//   phi(l) = (sqrt((M-1)/(a+l)) - sqrt(beta)) / l = -sqrt(beta) / (a s (1+s)),
//   s = sqrt(1 + l/a)   (cancellation-free, finite at l = 0),
// and x_m^a = x_bar + sqrt(beta) dX_m + dX w_bar + (dX Z^T) U phi U^T Z_m.
//
// Nodes are grouped by their number of local observations; each group runs
// the kernel instance whose eigenproblem size N is the smallest instantiated
// even size >= its l, with 64/N nodes per wavefront (one segment of N lanes
// per node).  The node list of a group is passed in `nodes`.
#include "common.h"
#include "device_util.h"

namespace lbmletkf {
namespace {
using namespace dev;

// ---------------------------------------------------------------------------
// observation route: SEGS = 64 / N nodes per wavefront, eigenproblem Z Z^T
// ---------------------------------------------------------------------------
template <int N>
struct ObsLayout {
    static_assert(N >= 8 && N % 2 == 0, "eigenproblem size must be even and >= 8");
    static constexpr int SEGS = 64 / N;
    static constexpr int cmax(int x, int y) { return x > y ? x : y; }
    // Jacobi rows; stages one node's dX (9 x 64) before, holds E' after
    static constexpr int RS = RowStride<N>::value;
    static constexpr int kRows = cmax(cmax(SEGS * N * RS, 9 * 64), SEGS * 9 * N);
    // per segment 10 N doubles: B = dX Z^T as [9][N], later C as [N][10]
    static constexpr int kBC = SEGS * 10 * N;
    static constexpr int kVec = 4 * 64;  // cs|red during Jacobi; psi t, h, mean increment after
    static constexpr int kObs = 2 * SEGS * N + (SEGS * N + 1) / 2;  // sw, dt, q
    static constexpr int kXbar = SEGS * 9 + 1;
    static constexpr int total = kRows + kBC + kVec + kObs + kXbar;
};

template <int N, typename T>
__global__ __launch_bounds__(64) void analysis_obs_kernel(AnalysisParams p, const int* nodes,
                                                          int count, int max_sweeps) {
    T* __restrict__ fs = reinterpret_cast<T*>(p.f);
    using L = ObsLayout<N>;
    constexpr int SEGS = L::SEGS;
    extern __shared__ double lds[];
    double* rows = lds;                              // [SEGS][N][RS]
    constexpr int RS = L::RS;
    double* BC = rows + L::kRows;                    // [SEGS][10 N]
    double* vec = BC + L::kBC;                       // [4][64]
    double* sw = vec + L::kVec;                      // [SEGS][N]
    double* dt = sw + SEGS * N;                      // [SEGS][N]
    int* qx = reinterpret_cast<int*>(dt + SEGS * N); // [SEGS][N]
    double* xb = rows + L::kRows + L::kBC + L::kVec + L::kObs;  // [SEGS][9]
    double2* cs = reinterpret_cast<double2*>(vec);   // Jacobi only
    double* red = vec + 128;                         // Jacobi only
    double* pt = vec;                                // psi_c t_c
    double* hv = vec + 64;                           // h_j
    double* dmv = vec + 128;                         // [SEGS][9] dX w_bar

    const int lane = threadIdx.x;
    const int nx = p.nx, ny = p.ny, M = p.members;
    const int nz = p.nvar * p.lmax;
    const int item0 = xcd_remap(blockIdx.x, gridDim.x) * SEGS;
    const int seg = lane / N;
    const int i = lane - seg * N;
    const bool active = seg < SEGS;
    const int sbase = active ? seg * N : 0;
    const bool mem = lane < M;
    const int mchunk = (M + SEGS - 1) / SEGS;  // members per lane group in B

    // ---- phase A (one node at a time, lane = member): x_bar, dX, local
    //      observations and B = dX Z^T (rows of Z: sqrt(r_j) dY[q_j][:])
#pragma unroll 1
    for (int sg = 0; sg < SEGS; ++sg) {
        const bool valid = item0 + sg < count;
        const int node = valid ? nodes[item0 + sg] : 0;
        const int x = node % nx, y = node / nx;
        double dx[9];
#pragma unroll
        for (int a = 0; a < 9; ++a)
            dx[a] = (valid && mem) ? PopIO<T>::load(fs + slot(src_node(x, y, a, nx, ny), a, lane, M), a)
                                   : 0.0;
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            const double xbar = wave_sum(dx[a]) / M;
            dx[a] = mem ? dx[a] - xbar : 0.0;
            if (lane == 0) xb[sg * 9 + a] = xbar;
        }
        wave_lds_sync();
        if (lane < N) {
            int q = 0;
            double w = 0.0, d = 0.0;
            if (valid && lane < nz) {
                const int slot = lane / p.nvar, var = lane - slot * p.nvar;
                const int k = p.loc_pt[(size_t)node * p.lmax + slot];
                if (k >= 0) {
                    q = k * p.nvar + var;
                    w = sqrt(p.loc_g[(size_t)node * p.lmax + slot] * p.rinv[var]);
                    d = w * p.dvec[q];
                }
            }
            qx[sg * N + lane] = q;
            sw[sg * N + lane] = w;
            dt[sg * N + lane] = d;
        }
        // stage dX of this node ([a][m]) in the not yet used Jacobi rows area
#pragma unroll
        for (int a = 0; a < 9; ++a) rows[a * 64 + lane] = dx[a];
        wave_lds_sync();
        // lane (g, j): partial sum of B[a][j] over member group g
        double b[9];
#pragma unroll
        for (int a = 0; a < 9; ++a) b[a] = 0.0;
        if (active) {
            const double wj = sw[sg * N + i];
            if (wj != 0.0) {
                const double* yrow = p.dY + (size_t)qx[sg * N + i] * M;
                const int m0 = seg * mchunk;
                const int m1 = min(M, m0 + mchunk);
#pragma unroll 2
                for (int m = m0; m < m1; ++m) {
                    const double yv = yrow[m];
#pragma unroll
                    for (int a = 0; a < 9; ++a) b[a] += rows[a * 64 + m] * yv;
                }
            }
        }
        // combine the member groups in a fixed order (group 0 keeps the sum)
#pragma unroll
        for (int g = 1; g < SEGS; ++g) {
            const int src = i + g * N;
#pragma unroll
            for (int a = 0; a < 9; ++a) {
                const double v = __shfl(b[a], active ? src : lane, kWave);
                b[a] += (seg == 0) ? v : 0.0;
            }
        }
        if (lane < N) {
            const double wj = sw[sg * N + lane];
#pragma unroll
            for (int a = 0; a < 9; ++a) BC[sg * 10 * N + a * N + lane] = b[a] * wj;
        }
        wave_lds_sync();
    }

    // ---- phase B: S = Z Z^T = diag(sw) K diag(sw) on the local observations
    double S[N], U[N];
    {
        const double wi = active ? sw[sbase + i] : 0.0;
        const double* Krow = p.K + (size_t)(active ? qx[sbase + i] : 0) * p.nobs;
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const double wk = sw[sbase + k];
            S[k] = (wi != 0.0 && wk != 0.0) ? wi * wk * Krow[qx[sbase + k]] : 0.0;
            U[k] = (k == i && active) ? 1.0 : 0.0;
        }
    }

    // ---- phase C: eigendecomposition
    const int sweeps = jacobi_eig<N, SEGS>(S, U, rows, cs, red, lane, max_sweeps);
    if (sweeps > max_sweeps && lane == 0) atomicAdd(p.eig_fail, 1);

    // ---- phase D: eigenvalue functions, U to LDS, t = U^T d~, h = U psi t
    const double lam = extract_lane_entry<N>(S, i);
    const double sq = sqrt(1.0 + lam / p.a);
    const double psi = 1.0 / (p.a + lam);
    const double phi = -p.sqrt_beta / (p.a * sq * (1.0 + sq));
    wave_lds_sync();
    if (active) {
        double2* my = reinterpret_cast<double2*>(rows + (size_t)(sbase + i) * RS);
#pragma unroll
        for (int k = 0; k < N / 2; ++k) my[k] = make_double2(U[2 * k], U[2 * k + 1]);
    }
    wave_lds_sync();
    {
        double t = 0.0;
        if (active)
            for (int k = 0; k < N; ++k) t += rows[(size_t)(sbase + k) * RS + i] * dt[sbase + k];
        pt[lane] = active ? psi * t : 0.0;
    }
    wave_lds_sync();
    {
        double h = 0.0;
#pragma unroll
        for (int c = 0; c < N; ++c) h += U[c] * pt[sbase + c];
        hv[lane] = active ? h : 0.0;
    }
    // ---- phase E: e = (B U)[:, i]; mean increment dm = B h (lanes a < 9)
    double e[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) e[a] = 0.0;
    if (active) {
        const double* Bs = BC + seg * 10 * N;
        for (int k = 0; k < N; ++k) {
            const double ukc = rows[(size_t)(sbase + k) * RS + i];
#pragma unroll
            for (int a = 0; a < 9; ++a) e[a] += Bs[a * N + k] * ukc;
        }
    }
    wave_lds_sync();  // h visible
    // population a = i, i + N, ... of the mean increment (N may be < 9)
    double dm[2] = {0.0, 0.0};
    if (active) {
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int a = i + r * N;
            if (a < 9) {
                const double* Bs = BC + seg * 10 * N + a * N;
                for (int j = 0; j < N; ++j) dm[r] += Bs[j] * hv[sbase + j];
            }
        }
    }
    wave_lds_sync();  // all reads of U (rows) done
    if (active) {
#pragma unroll
        for (int a = 0; a < 9; ++a) rows[(seg * 9 + a) * N + i] = phi * e[a];  // E'
#pragma unroll
        for (int r = 0; r < 2; ++r)
            if (i + r * N < 9) dmv[seg * 9 + i + r * N] = dm[r];
    }
    wave_lds_sync();
    // ---- phase F: C = E' U^T (own row of U)
    double cj[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        double acc = 0.0;
        if (active) {
#pragma unroll
            for (int c = 0; c < N; ++c) acc += rows[(seg * 9 + a) * N + c] * U[c];
        }
        cj[a] = acc;
    }
    wave_lds_sync();  // all reads of B done (phase E) -- overwrite with C
    if (active) {
        double* Cj = BC + seg * 10 * N + i * 10;
#pragma unroll
        for (int a = 0; a < 9; ++a) Cj[a] = cj[a];
        Cj[9] = 0.0;
    }
    wave_lds_sync();

    // ---- phase G (one node at a time, lane = member): apply and store
#pragma unroll 1
    for (int sg = 0; sg < SEGS; ++sg) {
        if (item0 + sg >= count) break;
        const int node = nodes[item0 + sg];
        const int x = node % nx, y = node / nx;
        double acc[9];
#pragma unroll
        for (int a = 0; a < 9; ++a) acc[a] = 0.0;
        const double* Cs = BC + sg * 10 * N;
#pragma unroll 2
        for (int j = 0; j < N; ++j) {
            const double wj = sw[sg * N + j];
            const double z = (mem && wj != 0.0) ? wj * p.dY[(size_t)qx[sg * N + j] * M + lane] : 0.0;
            const double2* c2 = reinterpret_cast<const double2*>(Cs + j * 10);
#pragma unroll
            for (int h = 0; h < 5; ++h) {
                const double2 v = c2[h];
                acc[2 * h] += v.x * z;
                if (2 * h + 1 < 9) acc[2 * h + 1] += v.y * z;
            }
        }
        if (mem) {
#pragma unroll
            for (int a = 0; a < 9; ++a) {
                T* sp = fs + slot(src_node(x, y, a, nx, ny), a, lane, M);
                const double fa = PopIO<T>::load(sp, a);
                const double xbar = xb[sg * 9 + a];
                PopIO<T>::store(sp, a, xbar + p.sqrt_beta * (fa - xbar) + dmv[sg * 9 + a] + acc[a]);
            }
        }
    }
}

template <int N>
hipError_t launch_n(const AnalysisParams& p, const int* nodes, int count, hipStream_t s) {
    using L = ObsLayout<N>;
    const size_t bytes = (size_t)L::total * sizeof(double);
    const int blocks = (count + L::SEGS - 1) / L::SEGS;
    if (blocks == 0) return hipSuccess;
    if (p.storage == kStoreF32Dev)
        analysis_obs_kernel<N, float><<<blocks, 64, bytes, s>>>(p, nodes, count, 30);
    else
        analysis_obs_kernel<N, double><<<blocks, 64, bytes, s>>>(p, nodes, count, 30);
    return hipGetLastError();
}

}  // namespace

#define LBMLETKF_OBS_SIZES(X) X(8) X(10) X(12) X(14) X(16) X(18) X(20) X(22) X(24) X(26) \
    X(28) X(30) X(32) X(40) X(48) X(56) X(64)

int obs_size_for(int n) {
    const int sizes[] = {
#define X(v) v,
        LBMLETKF_OBS_SIZES(X)
#undef X
    };
    for (int v : sizes)
        if (n <= v) return v;
    return 0;
}

int obs_lds_bytes(int n) {
    switch (n) {
#define X(v) case v: return ObsLayout<v>::total * (int)sizeof(double);
        LBMLETKF_OBS_SIZES(X)
#undef X
        default: return 1 << 30;
    }
}

hipError_t launch_analysis_obs(const AnalysisParams& p, const int* nodes, int count, int n,
                               hipStream_t s) {
    switch (n) {
#define X(v) case v: return launch_n<v>(p, nodes, count, s);
        LBMLETKF_OBS_SIZES(X)
#undef X
        default: return hipErrorInvalidValue;
    }
}

}  // namespace lbmletkf
