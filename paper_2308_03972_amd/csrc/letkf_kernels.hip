// Observation, ensemble statistics and LETKF analysis kernels (Sec. 3,
// Sec. 3.2.1, Sec. 3.2.2) plus the cycle diagnostics (Sec. 4.3.1).
//
// Analysis per grid node xi (one wavefront per node, lane = member or
// matrix row):
//   local observations L(xi): points with Gaspari-Cohn weight g > 0 within
//     2 d_cut, each weighted r_q = g / sigma_q^2 (R_loc^-1 = G o R^-1);
//   Z = R_loc^-1/2 dY restricted to L (l x M), d~ = R_loc^-1/2 (y^o - y_bar);
//   ensemble route (n = M): A = (M-1)/beta I + Z^T Z = U Lambda U^T,
//     w_bar = U Lambda^-1 U^T Z^T d~, dW = U sqrt((M-1) Lambda^-1) U^T;
//   observation route (n = l): Z Z^T = U Lambda U^T.  The M x M matrix then
//     has eigenvalues a + lambda_i (a = (M-1)/beta) on span(Z^T U) and a on
//     its complement, so  w_bar = Z^T U (a + Lambda)^-1 U^T d~  and
//     dW = sqrt(beta) I + Z^T U phi(Lambda) U^T Z with
//     phi(l) = (sqrt((M-1)/(a+l)) - sqrt(beta)) / l
//            = -sqrt(beta) / (a s (1 + s)),  s = sqrt(1 + l/a)
//     (the second form has no cancellation and is finite at l = 0);
//   x_m^a = x_bar + dX (w_bar + dW[:, m]) for the nine populations.
// The n x n symmetric eigenproblem is solved by parallel cyclic Jacobi
// (Golub & Van Loan, Sec. 8.5) with the Brent-Luk ordering: lane i holds row
// i of the matrix and of the eigenvector matrix in registers; each round
// rotates the neighbour pairs (2k+p, 2k+p+1) and swaps them, so two fixed
// pairings alternate and every pair meets once per n rounds.
#include <mutex>
#include <type_traits>

#include "common.h"
#include "device_util.h"

// Device scratch of the allocation-free diagnostics entry point: the per-block
// partial records of diag_partial_kernel.  Every GPU the library runs on holds
// its own copy until the process ends; all calls on one GPU share it.
static __device__ __align__(256) double scratch[lbmletkf::kStaticScratchBytes / sizeof(double)];

namespace lbmletkf {
namespace {
using namespace dev;

// ---------------------------------------------------------------------------
// observation operator: yf[m][nvar*k + var]
// ---------------------------------------------------------------------------
template <typename T>
__global__ void observe_kernel(const T* __restrict__ f, const int* __restrict__ pts, int npts,
                               int nvar, double* __restrict__ yf, int nx, int ny, int members) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= npts * members) return;
    const int k = t / members, m = t - k * members;  // members fastest: contiguous loads
    const int x = pts[2 * k], y = pts[2 * k + 1];
    double rho = 0.0, jx = 0.0, jy = 0.0;
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const double fa = PopIO<T>::load(f + slot(src_node(x, y, a, nx, ny), a, m, members), a);
        rho += fa;
        jx += cx_of(a) * fa;
        jy += cy_of(a) * fa;
    }
    double* o = yf + (size_t)m * npts * nvar + (size_t)k * nvar;
    if (nvar == 3) {
        o[0] = rho;
        o[1] = jx / rho;
        o[2] = jy / rho;
    } else {
        o[0] = jx / rho;
        o[1] = jy / rho;
    }
}

// ---------------------------------------------------------------------------
// observation-space statistics: y_bar, dY[q][m], d = y^o - y_bar
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void obs_stats_kernel(
    const double* __restrict__ yf, const double* __restrict__ yo, int nobs, int members,
    double* __restrict__ ybar, double* __restrict__ dY, double* __restrict__ dvec) {
    // one wavefront per observation q, lane = member
    const int q = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int m = threadIdx.x & 63;
    if (q >= nobs) return;
    const double v = m < members ? yf[(size_t)m * nobs + q] : 0.0;
    const double mean = wave_sum(v) / members;
    if (m < members) dY[(size_t)q * members + m] = v - mean;
    if (m == 0) {
        ybar[q] = mean;
        dvec[q] = yo[q] - mean;
    }
}

// K = dY dY^T (unweighted observation-space Gram matrix, nobs x nobs, inner
// dimension the members): the dense contraction under every node's
// Z Z^T = diag(sqrt r) K_L diag(sqrt r), on the matrix cores.  One wavefront
// per 16 x 16 tile of K, the member dimension in steps of 4 through
// v_mfma_{f64,f32}_16x16x4 (lane l supplies A[l % 16][l / 16] =
// dY[q0 + l % 16][m0 + l / 16] and B[l / 16][l % 16] = dY[r0 + l % 16][m0 + l / 16];
// result register j < 4 of lane l holds D[l / 16 + 4 j][l % 16] for the FP64
// instruction and D[4 (l / 16) + j][l % 16] for the FP32 one, as measured on
// gfx950 with lane-numbered operands).  Only tiles on or above the
// diagonal are computed; each value is written to both (q, r) and (r, q), so K
// is exactly symmetric.  T = double: FP64 MFMA (FP64 storage); T = float: FP32
// MFMA on dY rounded to FP32, FP32 accumulation (the precision form).
typedef double double4v __attribute__((ext_vector_type(4)));
typedef float float4v __attribute__((ext_vector_type(4)));

// One 16 x 16 x 4 matrix-core product, D = A B + C, in the precision of T.
__device__ __forceinline__ double4v mfma16(double a, double b, double4v c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ float4v mfma16(float a, float b, float4v c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
// Row of D held in result register j of lane l (column l % 16): FP64 and FP32
// instructions spread the rows differently.
template <typename T>
__device__ __forceinline__ int mfma16_row(int lane, int j) {
    return sizeof(T) == 8 ? (lane >> 4) + 4 * j : 4 * (lane >> 4) + j;
}

template <typename T>
__global__ __launch_bounds__(64) void obs_gram_kernel(const double* __restrict__ dY, int nobs,
                                                      int members, double* __restrict__ K) {
    const int tx = blockIdx.x, ty = blockIdx.y;
    if (ty > tx) return;  // uniform over the wavefront
    const int lane = threadIdx.x;
    const int i = lane & 15, kq = lane >> 4;
    const int qa = ty * 16 + i, rb = tx * 16 + i;
    const bool qin = qa < nobs, rin = rb < nobs;
    const double* arow = dY + (size_t)(qin ? qa : 0) * members;
    const double* brow = dY + (size_t)(rin ? rb : 0) * members;
    double out[4];
    if constexpr (sizeof(T) == 8) {
        double4v acc = {0.0, 0.0, 0.0, 0.0};
        for (int m0 = 0; m0 < members; m0 += 4) {
            const int m = m0 + kq;
            const double a = (qin && m < members) ? arow[m] : 0.0;
            const double b = (rin && m < members) ? brow[m] : 0.0;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) out[j] = acc[j];
    } else {
        float4v acc = {0.0f, 0.0f, 0.0f, 0.0f};
        for (int m0 = 0; m0 < members; m0 += 4) {
            const int m = m0 + kq;
            const float a = (qin && m < members) ? (float)arow[m] : 0.0f;
            const float b = (rin && m < members) ? (float)brow[m] : 0.0f;
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) out[j] = (double)acc[j];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int row = ty * 16 + mfma16_row<T>(lane, j), col = tx * 16 + i;
        if (row >= nobs || col >= nobs || (tx == ty && row > col)) continue;
        K[(size_t)row * nobs + col] = out[j];
        K[(size_t)col * nobs + row] = out[j];
    }
}

// ---------------------------------------------------------------------------
// local-observation table (static for a fixed network)
// ---------------------------------------------------------------------------
__global__ void local_table_kernel(const int* __restrict__ pts, int npts, double d_cut, int lmax,
                                   int nx, int ny, int* __restrict__ loc_pt,
                                   double* __restrict__ loc_g, int* __restrict__ overflow) {
    const int node = blockIdx.x * blockDim.x + threadIdx.x;
    if (node >= nx * ny) return;
    const int x = node % nx, y = node / nx;
    const bool infinite = !(d_cut > 0.0) || isinf(d_cut);
    const double lim = 4.0 * d_cut * d_cut;
    int cnt = 0;
    for (int k = 0; k < npts; ++k) {
        int dx = abs(x - pts[2 * k]), dy = abs(y - pts[2 * k + 1]);
        dx = min(dx, nx - dx);
        dy = min(dy, ny - dy);
        const double r2 = (double)(dx * dx + dy * dy);
        double g;
        if (infinite) {
            g = 1.0;
        } else {
            if (!(r2 < lim)) continue;
            // the polynomial vanishes at d = 2 d_cut; just inside, its rounding can
            // fall ~1e-16 below zero: the weight is kept non-negative
            g = fmax(gaspari_cohn(sqrt(r2) / d_cut), 0.0);
        }
        if (cnt < lmax) {
            loc_pt[(size_t)node * lmax + cnt] = k;
            loc_g[(size_t)node * lmax + cnt] = g;
        } else {
            atomicAdd(overflow, 1);
        }
        ++cnt;
    }
    for (int c = cnt; c < lmax; ++c) {
        loc_pt[(size_t)node * lmax + c] = -1;
        loc_g[(size_t)node * lmax + c] = 0.0;
    }
}

// ---------------------------------------------------------------------------
// ensemble route: one node per wavefront, eigenproblem (M-1)/beta I + Z^T Z
// (lane = member; sizes above M are padded with isolated (M-1)/beta rows)
// ---------------------------------------------------------------------------
// Nodes per wavefront of the ensemble route: N in {8, 16, 32} packs 64 / N
// nodes (a segment of N lanes each, N a power of two so that segment sums are
// xor shuffles inside the segment); 24, 48 and 64 take one node per wavefront.
__host__ __device__ constexpr int ens_segs(int n) { return (n == 8 || n == 16 || n == 32) ? 64 / n : 1; }

__host__ __device__ inline int ens_lds_doubles(int n, int nz) {
    const int segs = ens_segs(n);
    const int nzp = (nz + 1) & ~1;
    const int rs = (n % 4 == 2) ? n : n + 2;
    return 9 * 64 + segs * n * rs + 4 * 64 + 9 * n * segs + 64 + segs * (2 * nzp + nzp / 2) + 1;
}

// Sum over the aligned group of G lanes (G a power of two dividing 64).
template <int G>
__device__ __forceinline__ double group_sum(double v) {
    return group_reduce<G>(v, OpAdd());
}

// Z^T Z of the SEGS nodes of a wavefront on the matrix cores (N a multiple of
// 16): Z = R_loc^-1/2 dY restricted to each node's local observations (nz x M,
// members padded with zeros to N).  Per node the N x N product is NB x NB tiles
// of 16 x 16 (NB = N / 16), of which the NB (NB + 1) / 2 on or above the
// diagonal are accumulated over the observations in steps of 4 (lane l loads
// Z[j0 + l / 16][16 b + l % 16] once per member block b and feeds it as both
// operands: A = Z^T and B = Z carry the same numbers); the tiles go to the
// segment's rows in LDS, mirrored, and lane i of each segment returns row i of
// a I + Z^T Z.  MT: the matrix-core precision (double: FP64 MFMA; float: FP32
// MFMA with FP32 accumulation).  `obs` points at segment 0's weights, innovations
// and observation indices; segment s's are `seg_stride` doubles further.
template <int N, int SEGS, typename MT>
__device__ __forceinline__ void ens_gram_mfma(const AnalysisParams& p, const double* obs,
                                              int seg_stride, int nzp, int nz, double* rows,
                                              int lane, int seg, int i, double (&S)[N]) {
    static_assert(N % 16 == 0, "matrix-core tiles of 16");
    constexpr int NB = N / 16;
    constexpr int NT = NB * (NB + 1) / 2;
    constexpr int RS = RowStride<N>::value;
    using Acc = typename std::conditional<sizeof(MT) == 8, double4v, float4v>::type;
    const int M = p.members;
    const int kq = lane >> 4, c = lane & 15;
    Acc acc[SEGS][NT];
#pragma unroll
    for (int s = 0; s < SEGS; ++s)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[s][t] = Acc{0, 0, 0, 0};
    for (int j0 = 0; j0 < nz; j0 += 4) {
        const int jj = j0 + kq;
        const bool jin = jj < nz;
#pragma unroll
        for (int s = 0; s < SEGS; ++s) {
            const double* sw_s = obs + (size_t)s * seg_stride;
            const int* qx_s = reinterpret_cast<const int*>(sw_s + 2 * nzp);
            const double w = jin ? sw_s[jj] : 0.0;
            const double* yrow = p.dY + (size_t)(jin ? qx_s[jj] : 0) * M;
            // unconditional loads (member 0 past the ensemble), selected afterwards
            double y[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) y[b] = yrow[16 * b + c < M ? 16 * b + c : 0];
            MT z[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) z[b] = (MT)((jin && 16 * b + c < M) ? w * y[b] : 0.0);
            int t = 0;
#pragma unroll
            for (int I = 0; I < NB; ++I)
#pragma unroll
                for (int J = I; J < NB; ++J) {
                    acc[s][t] = mfma16(z[I], z[J], acc[s][t]);
                    ++t;
                }
        }
    }
    wave_lds_sync();
#pragma unroll
    for (int s = 0; s < SEGS; ++s) {
        double* rs = rows + (size_t)s * N * RS;
        int t = 0;
#pragma unroll
        for (int I = 0; I < NB; ++I)
#pragma unroll
            for (int J = I; J < NB; ++J, ++t)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int R = 16 * I + mfma16_row<MT>(lane, j), C = 16 * J + c;
                    if (I == J && R > C) continue;
                    const double v = (double)acc[s][t][j];
                    rs[(size_t)R * RS + C] = v;
                    rs[(size_t)C * RS + R] = v;
                }
    }
    wave_lds_sync();
    const double* mine = rows + (size_t)(seg < SEGS ? seg : 0) * N * RS;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const double v = (seg < SEGS && i < N) ? mine[(size_t)i * RS + k] : 0.0;
        S[k] = (k == i) ? p.a + v : v;
    }
}

// One wavefront: nodes node0 .. node0 + SEGS - 1 (those < nx * ny) of one
// problem, a segment of G = 64 / SEGS lanes per node, lane i of a segment =
// member i; the segment's rows of A and U are its first N lanes.
template <int N, typename T>
__device__ __forceinline__ void ens_body(const AnalysisParams p, int node0) {
    constexpr int SEGS = ens_segs(N);
    constexpr int G = kWave / SEGS;
    T* __restrict__ fs = reinterpret_cast<T*>(p.f);
    extern __shared__ double lds[];
    const int lane = threadIdx.x;
    const int nx = p.nx, ny = p.ny, M = p.members;
    const int plane = nx * ny;
    const int nz = p.nvar * p.lmax;
    const int nzp = (nz + 1) & ~1;
    double* sdx = lds;                   // [9][64]
    constexpr int RS = RowStride<N>::value;
    double* rows = sdx + 9 * 64;         // [SEGS][N][RS]  Jacobi rows, then U
    double* vec = rows + SEGS * N * RS;  // [4][64]
    double* se = vec + 4 * 64;           // [SEGS][9][N]
    double* zr = se + 9 * N * SEGS;      // [64]
    const int seg = lane / G;
    const int i = lane - seg * G;        // member
    const int sbase = seg * G;           // first lane of the segment
    double* sw = zr + 64 + seg * (2 * nzp + nzp / 2);  // this node's [nz] weights
    double* dt = sw + nzp;                             // [nz] scaled innovations
    int* qx = reinterpret_cast<int*>(dt + nzp);        // [nz] observation indices
    double2* cs = reinterpret_cast<double2*>(vec);
    double* red = vec + 128;
    const int node = node0 + seg;
    const bool here = node < plane;
    const int x = here ? node % nx : 0, y = here ? node / nx : 0;
    const bool mem = here && i < M;

    double fv[9], xbar[9];
    // unconditional loads (a lane past the ensemble or the grid reads member 0
    // of node 0 and discards it), so that the nine are in flight together
    const int mi = mem ? i : 0;
#pragma unroll
    for (int a = 0; a < 9; ++a)
        fv[a] = PopIO<T>::load(fs + slot(src_node(x, y, a, nx, ny), a, mi, M), a);
#pragma unroll
    for (int a = 0; a < 9; ++a) fv[a] = mem ? fv[a] : 0.0;
    if (p.diag_node && here)
        node_diag_record<G>(fv, mem, M, node, plane, p.truth_uv,
                            p.diag_node + (size_t)node * kDiagFieldCount);
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        xbar[a] = group_sum<G>(fv[a]) / M;
        sdx[a * 64 + lane] = mem ? fv[a] - xbar[a] : 0.0;
    }
    for (int j = i; j < nz; j += G) {
        const int slot_ = j / p.nvar, var = j - slot_ * p.nvar;
        const int k = here ? p.loc_pt[(size_t)node * p.lmax + slot_] : -1;
        const int q = k >= 0 ? k * p.nvar + var : 0;
        const double w = k >= 0 ? sqrt(p.loc_g[(size_t)node * p.lmax + slot_] * p.rinv[var]) : 0.0;
        qx[j] = q;
        sw[j] = w;
        dt[j] = w * p.dvec[q];
    }
    wave_lds_sync();
    // A = a I + Z^T Z and g = Z^T d~
    double S[N], U[N];
    double g = 0.0;
    constexpr int kZc = 8;
    if constexpr (N % 16 == 0) {
        // Z^T Z on the matrix cores (FP64 MFMA for FP64 storage, FP32 MFMA for
        // the precision form), g on the vector units
        ens_gram_mfma<N, SEGS, T>(p, zr + 64, 2 * nzp + nzp / 2, nzp, nz, rows, lane, seg, i, S);
        for (int j0 = 0; j0 < nz; j0 += kZc) {
            double zc[kZc];
#pragma unroll
            for (int t = 0; t < kZc; ++t)
                zc[t] = p.dY[(size_t)qx[min(j0 + t, nz - 1)] * M + (mem ? i : 0)];
#pragma unroll
            for (int t = 0; t < kZc; ++t) {
                const int j = j0 + t;
                if (j >= nz) break;  // uniform over the wavefront
                g += (mem ? sw[j] * zc[t] : 0.0) * dt[j];
            }
        }
    } else {
#pragma unroll
    for (int k = 0; k < N; ++k) S[k] = (k == i) ? p.a : 0.0;
    // the perturbations are loaded eight observations at a time, unconditionally
    // (a non-member lane reads member 0), so that the loads of a chunk are in
    // flight together; the sums run in observation order
    for (int j0 = 0; j0 < nz; j0 += kZc) {
        double zc[kZc];
#pragma unroll
        for (int t = 0; t < kZc; ++t)
            zc[t] = p.dY[(size_t)qx[min(j0 + t, nz - 1)] * M + (mem ? i : 0)];
#pragma unroll
        for (int t = 0; t < kZc; ++t) {
            const int j = j0 + t;
            if (j >= nz) break;  // uniform over the wavefront
            const double z = mem ? sw[j] * zc[t] : 0.0;
            g += z * dt[j];
            wave_lds_sync();
            zr[lane] = z;
            wave_lds_sync();
#pragma unroll
            for (int k = 0; k < N; ++k) S[k] += z * zr[sbase + k];
        }
    }
    }
#pragma unroll
    for (int k = 0; k < N; ++k) U[k] = (k == i) ? 1.0 : 0.0;
    const int sweeps = jacobi_eig<N, SEGS>(S, U, rows, cs, red, lane, p.max_sweeps);
    if (sweeps > p.max_sweeps && lane == 0) atomicAdd(p.eig_fail, 1);
    const double lam = extract_lane_entry<N>(S, i);
    const double psi = i < N ? 1.0 / lam : 0.0;
    const double mu = i < N ? sqrt((M - 1) / lam) : 0.0;
    double* gv = vec;        // g
    wave_lds_sync();
    gv[lane] = g;
    if (i < N) {
        double2* my = reinterpret_cast<double2*>(rows + (size_t)(seg * N + i) * RS);
#pragma unroll
        for (int k = 0; k < N / 2; ++k) my[k] = make_double2(U[2 * k], U[2 * k + 1]);
    }
    wave_lds_sync();
    double t = 0.0;
    double e[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) e[a] = 0.0;
    if (i < N) {
        for (int k = 0; k < N; ++k) {
            const double ukc = rows[(size_t)(seg * N + k) * RS + i];
            t += ukc * gv[sbase + k];
#pragma unroll
            for (int a = 0; a < 9; ++a) e[a] += sdx[a * 64 + sbase + k] * ukc;
        }
    }
    double dmean[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) dmean[a] = group_sum<G>(i < N ? e[a] * psi * t : 0.0);
    if (i < N) {
#pragma unroll
        for (int a = 0; a < 9; ++a) se[(seg * 9 + a) * N + i] = e[a] * mu;
    }
    wave_lds_sync();
    double xa[9];  // the analysis as stored (diagnostics)
#pragma unroll
    for (int a = 0; a < 9; ++a) xa[a] = 0.0;
    if (mem) {
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            double acc = 0.0;
#pragma unroll
            for (int c = 0; c < N; ++c) acc += se[(seg * 9 + a) * N + c] * U[c];
            const double v = xbar[a] + dmean[a] + acc;
            PopIO<T>::store(fs + slot(src_node(x, y, a, nx, ny), a, i, M), a, v);
            xa[a] = PopIO<T>::round(v, a);
        }
    }
    if (p.diag_node && here)
        node_diag_record<G>(xa, mem, M, node, plane, p.truth_uv,
                            p.diag_node + ((size_t)plane + node) * kDiagFieldCount);
}

template <int N, typename T>
__global__ __launch_bounds__(64) void analysis_ens_kernel(AnalysisParams p) {
    const int node0 = xcd_remap(blockIdx.x, gridDim.x) * ens_segs(N);
    if (node0 >= p.nx * p.ny) return;
    ens_body<N, T>(p, node0);
}

// Batched form: wavefront w takes waves[w] = (problem, node).
template <int N, typename T>
__global__ __launch_bounds__(64) void analysis_ens_batch_kernel(const AnalysisParams* P,
                                                                const int2* waves, int nwaves) {
    const int w = xcd_remap(blockIdx.x, gridDim.x);
    if (w >= nwaves) return;
    const int2 d = waves[w];  // (problem, first node of the wavefront's ens_segs(N) nodes)
    ens_body<N, T>(P[d.x], d.y);
}

// ---------------------------------------------------------------------------
// diagnostics: RMSE of the ensemble-mean velocity, spread, non-finite count,
// density range.  Deterministic two-pass reduction.
// ---------------------------------------------------------------------------
constexpr int kDiagBlock = 256;
constexpr int kDiagWaves = kDiagBlock / kWave;
constexpr int kDiagNodes = 64;  // nodes per block: 16 per wavefront, lane = member
constexpr int kDiagFields = 5;  // err2, spread2, nonfinite, rho_min, rho_max

template <typename T>
__global__ __launch_bounds__(kDiagBlock) void diag_partial_kernel(
    const T* __restrict__ f, const double* __restrict__ truth_uv, int nx, int ny, int members,
    double* __restrict__ partial) {
    const int plane = nx * ny;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int nodes_per_wave = kDiagNodes / kDiagWaves;
    double err2 = 0.0, spr2 = 0.0, bad = 0.0, rmin = INFINITY, rmax = -INFINITY;
    for (int k = 0; k < nodes_per_wave; ++k) {
        const int i = blockIdx.x * kDiagNodes + wave * nodes_per_wave + k;
        if (i >= plane) break;
        const int y = i / nx, x = i - y * nx;
        double u = 0.0, v = 0.0, rho = 1.0;
        if (lane < members) {
            double jx = 0.0, jy = 0.0;
            rho = 0.0;
#pragma unroll
            for (int a = 0; a < 9; ++a) {
                const double fa =
                    PopIO<T>::load(f + slot(src_node(x, y, a, nx, ny), a, lane, members), a);
                rho += fa;
                jx += cx_of(a) * fa;
                jy += cy_of(a) * fa;
            }
            u = jx / rho;
            v = jy / rho;
            if (!isfinite(rho) || !isfinite(u) || !isfinite(v)) bad += 1.0;
            rmin = fmin(rmin, rho);
            rmax = fmax(rmax, rho);
        }
        const double ub = wave_sum(u) / members, vb = wave_sum(v) / members;
        if (truth_uv && lane == 0) {
            const double du = ub - truth_uv[i], dv = vb - truth_uv[plane + i];
            err2 += du * du + dv * dv;
        }
        if (members > 1) {
            const double du = lane < members ? u - ub : 0.0, dv = lane < members ? v - vb : 0.0;
            const double s2 = wave_sum(du * du + dv * dv);
            if (lane == 0) spr2 += s2 / (members - 1);
        }
    }
    // combine: lanes of each wave, then the waves in a fixed order
    bad = wave_sum(bad);
    rmin = group_reduce<kWave>(rmin, OpMin());
    rmax = group_reduce<kWave>(rmax, OpMax());
    __shared__ double red[kDiagFields][kDiagWaves];
    if (lane == 0) {
        red[0][wave] = err2;
        red[1][wave] = spr2;
        red[2][wave] = bad;
        red[3][wave] = rmin;
        red[4][wave] = rmax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double acc[kDiagFields] = {0.0, 0.0, 0.0, INFINITY, -INFINITY};
        for (int w = 0; w < kDiagWaves; ++w) {
            acc[0] += red[0][w];
            acc[1] += red[1][w];
            acc[2] += red[2][w];
            acc[3] = fmin(acc[3], red[3][w]);
            acc[4] = fmax(acc[4], red[4][w]);
        }
        for (int k = 0; k < kDiagFields; ++k) partial[(size_t)blockIdx.x * kDiagFields + k] = acc[k];
    }
}

// Per-node records (diagnostics folded into the analysis): block (b, s)
// reduces records [b * kDiagBlock, (b + 1) * kDiagBlock) of state s (0
// forecast, 1 analysis) in a fixed tree order into partial[s][b].
__global__ __launch_bounds__(kDiagBlock) void diag_fold_kernel(const double* __restrict__ rec,
                                                               int plane,
                                                               double* __restrict__ partial) {
    __shared__ double red[kDiagFields][kDiagBlock];
    const int t = threadIdx.x;
    const int i = blockIdx.x * kDiagBlock + t;
    const double* r = rec + ((size_t)blockIdx.y * plane + i) * kDiagFields;
    const bool in = i < plane;
    red[0][t] = in ? r[0] : 0.0;
    red[1][t] = in ? r[1] : 0.0;
    red[2][t] = in ? r[2] : 0.0;
    red[3][t] = in ? r[3] : INFINITY;
    red[4][t] = in ? r[4] : -INFINITY;
    __syncthreads();
    for (int s = kDiagBlock / 2; s > 0; s >>= 1) {
        if (t < s) {
            red[0][t] += red[0][t + s];
            red[1][t] += red[1][t + s];
            red[2][t] += red[2][t + s];
            red[3][t] = fmin(red[3][t], red[3][t + s]);
            red[4][t] = fmax(red[4][t], red[4][t + s]);
        }
        __syncthreads();
    }
    if (t == 0) {
        double* o = partial + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * kDiagFields;
        for (int k = 0; k < kDiagFields; ++k) o[k] = red[k][0];
    }
}

__global__ __launch_bounds__(kDiagBlock) void diag_final_kernel(const double* __restrict__ partial,
                                                                int nblocks, int plane,
                                                                double* __restrict__ out) {
    __shared__ double red[kDiagFields][kDiagBlock];
    double err2 = 0.0, spr2 = 0.0, bad = 0.0, rmin = INFINITY, rmax = -INFINITY;
    for (int b = threadIdx.x; b < nblocks; b += kDiagBlock) {
        err2 += partial[b * kDiagFields + 0];
        spr2 += partial[b * kDiagFields + 1];
        bad += partial[b * kDiagFields + 2];
        rmin = fmin(rmin, partial[b * kDiagFields + 3]);
        rmax = fmax(rmax, partial[b * kDiagFields + 4]);
    }
    red[0][threadIdx.x] = err2;
    red[1][threadIdx.x] = spr2;
    red[2][threadIdx.x] = bad;
    red[3][threadIdx.x] = rmin;
    red[4][threadIdx.x] = rmax;
    __syncthreads();
    for (int s = kDiagBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            red[0][threadIdx.x] += red[0][threadIdx.x + s];
            red[1][threadIdx.x] += red[1][threadIdx.x + s];
            red[2][threadIdx.x] += red[2][threadIdx.x + s];
            red[3][threadIdx.x] = fmin(red[3][threadIdx.x], red[3][threadIdx.x + s]);
            red[4][threadIdx.x] = fmax(red[4][threadIdx.x], red[4][threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = sqrt(red[0][0] / plane);
        out[1] = sqrt(red[1][0] / plane);
        out[2] = red[2][0];
        out[3] = red[3][0];
        out[4] = red[4][0];
        out[5] = 0.0;
        out[6] = 0.0;
        out[7] = 0.0;
    }
}

__global__ void synth_obs_kernel(const double* __restrict__ y, const double* __restrict__ eps,
                                 const double* __restrict__ sigma, double* __restrict__ yo,
                                 int n) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) yo[q] = y[q] + sigma[q] * eps[q];
}

template <int N, typename T>
hipError_t launch_ens_t(const AnalysisParams& p, hipStream_t s) {
    const size_t bytes = (size_t)ens_lds_doubles(N, p.nvar * p.lmax) * sizeof(double);
    const int plane = p.nx * p.ny;
    if (bytes > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)analysis_ens_kernel<N, T>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)bytes);
        if (e != hipSuccess) return e;
    }
    analysis_ens_kernel<N, T><<<(plane + ens_segs(N) - 1) / ens_segs(N), 64, bytes, s>>>(p);
    return hipGetLastError();
}

template <int N>
hipError_t launch_ens(const AnalysisParams& p, hipStream_t s) {
    return p.storage == kStoreF32Dev ? launch_ens_t<N, float>(p, s) : launch_ens_t<N, double>(p, s);
}

hipError_t launch_ens_sized(const AnalysisParams& p, int n, hipStream_t s) {
    switch (n) {
        case 8: return launch_ens<8>(p, s);
        case 16: return launch_ens<16>(p, s);
        case 24: return launch_ens<24>(p, s);
        case 32: return launch_ens<32>(p, s);
        case 48: return launch_ens<48>(p, s);
        case 64: return launch_ens<64>(p, s);
        default: return hipErrorInvalidValue;
    }
}

template <int N, typename T>
hipError_t launch_ens_batch_t(const AnalysisParams* P, const int2* waves, int nwaves, int nz_max,
                              hipStream_t s) {
    if (nwaves == 0) return hipSuccess;
    const size_t bytes = (size_t)ens_lds_doubles(N, nz_max) * sizeof(double);
    if (bytes > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)analysis_ens_batch_kernel<N, T>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)bytes);
        if (e != hipSuccess) return e;
    }
    analysis_ens_batch_kernel<N, T><<<nwaves, 64, bytes, s>>>(P, waves, nwaves);
    return hipGetLastError();
}

template <int N>
hipError_t launch_ens_batch(const AnalysisParams* P, const int2* waves, int nwaves, int nz_max,
                            int storage, hipStream_t s) {
    return storage == kStoreF32Dev ? launch_ens_batch_t<N, float>(P, waves, nwaves, nz_max, s)
                                   : launch_ens_batch_t<N, double>(P, waves, nwaves, nz_max, s);
}

}  // namespace

hipError_t launch_analysis_ens_batch(const AnalysisParams* d_params, const int2* d_waves,
                                     int nwaves, int n, int nz_max, int storage, hipStream_t s) {
    switch (n) {
        case 8: return launch_ens_batch<8>(d_params, d_waves, nwaves, nz_max, storage, s);
        case 16: return launch_ens_batch<16>(d_params, d_waves, nwaves, nz_max, storage, s);
        case 24: return launch_ens_batch<24>(d_params, d_waves, nwaves, nz_max, storage, s);
        case 32: return launch_ens_batch<32>(d_params, d_waves, nwaves, nz_max, storage, s);
        case 48: return launch_ens_batch<48>(d_params, d_waves, nwaves, nz_max, storage, s);
        case 64: return launch_ens_batch<64>(d_params, d_waves, nwaves, nz_max, storage, s);
        default: return hipErrorInvalidValue;
    }
}

int ens_size_for(int n) {
    const int sizes[] = {8, 16, 24, 32, 48, 64};
    for (int v : sizes)
        if (n <= v) return v;
    return 0;
}

int ens_lds_bytes(int n, int nz) { return ens_lds_doubles(n, nz) * (int)sizeof(double); }

int ens_segments(int n) { return ens_segs(n); }

hipError_t launch_observe(const void* f, const int* pts, int npts, int nvar, double* yf,
                          LbmDims d, int storage, hipStream_t s) {
    const int total = npts * d.members;
    if (storage == kStoreF32Dev)
        observe_kernel<float><<<(total + 255) / 256, 256, 0, s>>>((const float*)f, pts, npts, nvar,
                                                                   yf, d.nx, d.ny, d.members);
    else
        observe_kernel<double><<<(total + 255) / 256, 256, 0, s>>>((const double*)f, pts, npts,
                                                                    nvar, yf, d.nx, d.ny, d.members);
    return hipGetLastError();
}

hipError_t launch_obs_stats(const double* yf, const double* yo, int nobs, int members,
                            double* ybar, double* dY, double* dvec, double* K, int storage,
                            hipStream_t s) {
    obs_stats_kernel<<<(nobs + 3) / 4, 256, 0, s>>>(yf, yo, nobs, members, ybar, dY, dvec);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !K) return e;
    const int tiles = (nobs + 15) / 16;
    if (storage == kStoreF32Dev)
        obs_gram_kernel<float><<<dim3(tiles, tiles), 64, 0, s>>>(dY, nobs, members, K);
    else
        obs_gram_kernel<double><<<dim3(tiles, tiles), 64, 0, s>>>(dY, nobs, members, K);
    return hipGetLastError();
}

hipError_t launch_local_table(const int* pts, int npts, double d_cut, int lmax, int nx, int ny,
                              int* loc_pt, double* loc_g, int* overflow, hipStream_t s) {
    const int plane = nx * ny;
    local_table_kernel<<<(plane + 255) / 256, 256, 0, s>>>(pts, npts, d_cut, lmax, nx, ny, loc_pt,
                                                            loc_g, overflow);
    return hipGetLastError();
}

hipError_t launch_analysis_ens(const AnalysisParams& p, int n, hipStream_t s) {
    return launch_ens_sized(p, n, s);
}

int diag_blocks_for(int plane) { return (plane + kDiagNodes - 1) / kDiagNodes; }

size_t diag_partial_bytes(int plane) {
    return (size_t)diag_blocks_for(plane) * kDiagFields * sizeof(double);
}

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_addr[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch(void** addr) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_addr[dev]) {
        // the array's device address on the current device (its host-side name
        // is not a device pointer)
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_addr[dev] = p;
    }
    *addr = g_scratch_addr[dev];
    return hipSuccess;
}

hipError_t launch_diag(const void* f, const double* truth_uv, LbmDims d, int storage,
                       double* partial, int nblocks, double* out, hipStream_t s) {
    const int need = diag_blocks_for(d.nx * d.ny);
    if (need > nblocks) return hipErrorInvalidValue;
    if (storage == kStoreF32Dev)
        diag_partial_kernel<float><<<need, kDiagBlock, 0, s>>>((const float*)f, truth_uv, d.nx, d.ny,
                                                               d.members, partial);
    else
        diag_partial_kernel<double><<<need, kDiagBlock, 0, s>>>((const double*)f, truth_uv, d.nx,
                                                                d.ny, d.members, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    diag_final_kernel<<<1, kDiagBlock, 0, s>>>(partial, need, d.nx * d.ny, out);
    return hipGetLastError();
}

int diag_fold_blocks(int plane) { return (plane + kDiagBlock - 1) / kDiagBlock; }

hipError_t launch_diag_nodes_final(const double* diag_node, int plane, double* partial,
                                   double* out_forecast, double* out_analysis, hipStream_t s) {
    static_assert(kDiagFields == kDiagFieldCount, "one diagnostics record layout");
    const int nb = diag_fold_blocks(plane);
    diag_fold_kernel<<<dim3(nb, 2), kDiagBlock, 0, s>>>(diag_node, plane, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    diag_final_kernel<<<1, kDiagBlock, 0, s>>>(partial, nb, plane, out_forecast);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    diag_final_kernel<<<1, kDiagBlock, 0, s>>>(partial + (size_t)nb * kDiagFields, nb, plane,
                                               out_analysis);
    return hipGetLastError();
}

hipError_t launch_synth_obs(const double* y, const double* eps, const double* sigma, double* yo,
                            int n, hipStream_t s) {
    synth_obs_kernel<<<(n + 255) / 256, 256, 0, s>>>(y, eps, sigma, yo, n);
    return hipGetLastError();
}

}  // namespace lbmletkf
