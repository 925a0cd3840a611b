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
#include "common.h"

namespace lbmletkf {
namespace {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Order this wave's LDS writes before its later LDS reads (cross-lane).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// Printed Gaspari-Cohn piecewise function, Horner form.
__device__ __forceinline__ double gaspari_cohn(double d) {
    if (d <= 1.0) {
        return (((((-0.25 * d + 0.5) * d + 0.625) * d - 5.0 / 3.0) * d) * d) + 1.0;
    }
    if (d < 2.0) {
        return ((((d / 12.0 - 0.5) * d + 0.625) * d + 5.0 / 3.0) * d - 5.0) * d + 4.0 -
               (2.0 / 3.0) / d;
    }
    return 0.0;
}

// ---------------------------------------------------------------------------
// observation operator: yf[m][nvar*k + var]
// ---------------------------------------------------------------------------
__global__ void observe_kernel(const double* __restrict__ f, const int* __restrict__ pts,
                               int npts, int nvar, double* __restrict__ yf, int nx, int ny,
                               int members) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= npts * members) return;
    const int m = t / npts, k = t - m * npts;
    const int x = pts[2 * k], y = pts[2 * k + 1];
    const size_t plane = (size_t)nx * ny;
    double rho = 0.0, jx = 0.0, jy = 0.0;
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const int xs = wrap(x - cx_of(a), nx), ys = wrap(y - cy_of(a), ny);
        const double fa = f[((size_t)m * 9 + a) * plane + (size_t)ys * nx + xs];
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
__global__ void obs_stats_kernel(const double* __restrict__ yf, const double* __restrict__ yo,
                                 int nobs, int members, double* __restrict__ ybar,
                                 double* __restrict__ dY, double* __restrict__ dvec) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nobs) return;
    double s = 0.0;
    for (int m = 0; m < members; ++m) s += yf[(size_t)m * nobs + q];
    const double mean = s / members;
    for (int m = 0; m < members; ++m) dY[(size_t)q * members + m] = yf[(size_t)m * nobs + q] - mean;
    ybar[q] = mean;
    dvec[q] = yo[q] - mean;
}

// K = dY dY^T (unweighted observation-space Gram matrix)
__global__ void obs_gram_kernel(const double* __restrict__ dY, int nobs, int members,
                                double* __restrict__ K) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nobs * nobs) return;
    const int q = t / nobs, r = t - q * nobs;
    const double* a = dY + (size_t)q * members;
    const double* b = dY + (size_t)r * members;
    double s = 0.0;
    for (int m = 0; m < members; ++m) s += a[m] * b[m];
    K[t] = s;
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
            g = gaspari_cohn(sqrt(r2) / d_cut);
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
// wave-level parallel Jacobi on an N x N symmetric matrix (N even, N <= 64)
// lane i < N holds row i of S and of U (U accumulates the rotations).
// ---------------------------------------------------------------------------
template <int N>
__device__ __forceinline__ double extract_lane_entry(const double (&R)[N], int col) {
    double v = 0.0;
#pragma unroll
    for (int r = 0; r < N; ++r) v = (r == col) ? R[r] : v;
    return v;
}

template <int N, int P>
__device__ __forceinline__ void jacobi_round(double (&S)[N], double (&U)[N], double* cs,
                                             int lane) {
    const bool first = ((lane - P) & 1) == 0;
    int partner = first ? lane + 1 : lane - 1;
    const bool paired = lane < N && partner >= 0 && partner < N;
    if (!paired) partner = lane;
    const double d_own = extract_lane_entry<N>(S, lane);
    const double e_own = extract_lane_entry<N>(S, partner);
    const double d_par = __shfl(d_own, partner, kWave);
    const double apq = __shfl(e_own, first ? lane : partner, kWave);  // from the first lane
    const double app = first ? d_own : d_par;
    const double aqq = first ? d_par : d_own;
    double c = 1.0, s = 0.0;
    if (paired && apq != 0.0) {
        const double theta = (aqq - app) / (2.0 * apq);
        double t = 1.0 / (fabs(theta) + sqrt(1.0 + theta * theta));
        if (theta < 0.0) t = -t;
        c = 1.0 / sqrt(1.0 + t * t);
        s = t * c;
    }
    // publish (c, s); the pair (r, r+1) is read from its first lane r
    wave_lds_sync();
    cs[2 * lane] = c;
    cs[2 * lane + 1] = s;
    wave_lds_sync();
    // columns: S <- S J P and U <- U J P (rotate, then swap the pair)
#pragma unroll
    for (int r = P; r + 1 < N; r += 2) {
        const double cr = cs[2 * r], sr = cs[2 * r + 1];
        const double a0 = S[r], a1 = S[r + 1];
        S[r] = sr * a0 + cr * a1;
        S[r + 1] = cr * a0 - sr * a1;
        const double u0 = U[r], u1 = U[r + 1];
        U[r] = sr * u0 + cr * u1;
        U[r + 1] = cr * u0 - sr * u1;
    }
    // rows: S <- P^T J^T S (rows of the pair exchanged across lanes)
    const double sg = first ? s : -s;
#pragma unroll
    for (int r = 0; r < N; ++r) {
        const double par = __shfl(S[r], partner, kWave);
        S[r] = c * par + sg * S[r];
    }
}

// Returns the number of sweeps used (max_sweeps + 1 if not converged).
template <int N>
__device__ int jacobi_eig(double (&S)[N], double (&U)[N], double* cs, int lane,
                          int max_sweeps) {
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        double off = 0.0, dg = 0.0;
#pragma unroll
        for (int r = 0; r < N; ++r) {
            const double v2 = S[r] * S[r];
            if (r == lane) dg += v2; else off += v2;
        }
        if (lane >= N) { off = 0.0; dg = 0.0; }
        off = wave_sum(off);
        dg = wave_sum(dg);
        if (off <= 1e-26 * dg) return sweep;
        for (int rr = 0; rr < N / 2; ++rr) {
            jacobi_round<N, 0>(S, U, cs, lane);
            jacobi_round<N, 1>(S, U, cs, lane);
        }
    }
    double off = 0.0, dg = 0.0;
#pragma unroll
    for (int r = 0; r < N; ++r) {
        const double v2 = S[r] * S[r];
        if (r == lane) dg += v2; else off += v2;
    }
    if (lane >= N) { off = 0.0; dg = 0.0; }
    off = wave_sum(off);
    dg = wave_sum(dg);
    return off <= 1e-26 * dg ? max_sweeps : max_sweeps + 1;
}

// ---------------------------------------------------------------------------
// per-node LETKF analysis; OBS selects the observation route
// ---------------------------------------------------------------------------
struct WaveLds {
    double* dx;    // [9][64]  forecast perturbations dX (zero for lanes >= M)
    double* u;     // [N][N+1] eigenvectors, row k = U[k][:]
    double* cs;    // [128]    rotation parameters
    double* psi;   // [64]
    double* phi;   // [64]
    double* rhs;   // [64]     route E: Z^T d~
    double* e;     // [9][N]
    double* b;     // [9][N]   route O: B = dX Z^T, then C = B U phi U^T
    double* zr;    // [64]     route E: one row of Z
    double* sw;    // [nzp]    sqrt(r_q)
    double* dt;    // [nzp]    d~
    int* q;        // [nzp]    observation index
};

__host__ __device__ inline int lds_doubles_per_wave(int n, int nz) {
    const int nzp = (nz + 1) & ~1;
    return 9 * 64 + n * (n + 1) + 128 + 3 * 64 + 2 * 9 * n + 64 + 2 * nzp + nzp / 2 + 1;
}

__device__ inline WaveLds carve(double* base, int n, int nz) {
    const int nzp = (nz + 1) & ~1;
    WaveLds w;
    w.dx = base;
    w.u = w.dx + 9 * 64;
    w.cs = w.u + n * (n + 1);
    w.psi = w.cs + 128;
    w.phi = w.psi + 64;
    w.rhs = w.phi + 64;
    w.e = w.rhs + 64;
    w.b = w.e + 9 * n;
    w.zr = w.b + 9 * n;
    w.sw = w.zr + 64;
    w.dt = w.sw + nzp;
    w.q = reinterpret_cast<int*>(w.dt + nzp);
    return w;
}

template <int N, bool OBS>
__global__ __launch_bounds__(64) void analysis_kernel(AnalysisParams p, int lds_per_wave,
                                                      int max_sweeps) {
    extern __shared__ double lds[];
    const int lane = threadIdx.x;
    const int node = blockIdx.x;
    const int nx = p.nx, ny = p.ny, M = p.members;
    const int plane = nx * ny;
    if (node >= plane) return;
    const int nz = p.nvar * p.lmax;
    WaveLds w = carve(lds, N, nz);
    const int x = node % nx, y = node / nx;
    const bool mem = lane < M;

    // ---- forecast ensemble at this node: canonical f_a from its storage slot
    double fv[9], xbar[9], dx[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const int xs = wrap(x - cx_of(a), nx), ys = wrap(y - cy_of(a), ny);
        fv[a] = mem ? p.f[((size_t)lane * 9 + a) * plane + (size_t)ys * nx + xs] : 0.0;
    }
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        xbar[a] = wave_sum(fv[a]) / M;
        dx[a] = mem ? fv[a] - xbar[a] : 0.0;
        w.dx[a * 64 + lane] = dx[a];
    }

    // ---- local observations, weights sqrt(g / sigma^2), scaled innovation
    for (int j = lane; j < nz; j += kWave) {
        const int slot = j / p.nvar, var = j - slot * p.nvar;
        const int k = p.loc_pt[(size_t)node * p.lmax + slot];
        const double g = p.loc_g[(size_t)node * p.lmax + slot];
        const int q = k >= 0 ? k * p.nvar + var : 0;
        const double sw = k >= 0 ? sqrt(g * p.rinv[var]) : 0.0;
        w.q[j] = q;
        w.sw[j] = sw;
        w.dt[j] = sw * p.dvec[q];
    }
    wave_lds_sync();

    // ---- the symmetric eigenproblem
    double S[N], U[N];
    if constexpr (OBS) {
        const bool row = lane < nz;
        const double swj = row ? w.sw[lane] : 0.0;
        const double* Krow = p.K + (size_t)(row ? w.q[lane] : 0) * p.nobs;
#pragma unroll
        for (int k = 0; k < N; ++k) {
            double v = 0.0;
            if (row && k < nz) v = swj * w.sw[k] * Krow[w.q[k]];
            S[k] = v;
            U[k] = (k == lane) ? 1.0 : 0.0;
        }
    } else {
#pragma unroll
        for (int k = 0; k < N; ++k) {
            S[k] = (k == lane) ? p.a : 0.0;
            U[k] = (k == lane) ? 1.0 : 0.0;
        }
        double g = 0.0;
        for (int j = 0; j < nz; ++j) {
            const double z = mem ? w.sw[j] * p.dY[(size_t)w.q[j] * M + lane] : 0.0;
            g += z * w.dt[j];
            wave_lds_sync();
            w.zr[lane] = z;
            wave_lds_sync();
#pragma unroll
            for (int k = 0; k < N; ++k) S[k] += z * w.zr[k];
        }
        w.rhs[lane] = g;
    }
    const int sweeps = jacobi_eig<N>(S, U, w.cs, lane, max_sweeps);
    if (sweeps > max_sweeps && lane == 0) atomicAdd(p.eig_fail, 1);

    // ---- eigenvalue functions and U in LDS
    const double lam = extract_lane_entry<N>(S, lane);
    double psi, phi;
    if constexpr (OBS) {
        const double s = sqrt(1.0 + lam / p.a);
        psi = 1.0 / (p.a + lam);
        phi = -p.sqrt_beta / (p.a * s * (1.0 + s));
    } else {
        psi = 1.0 / lam;
        phi = sqrt((M - 1) / lam);
    }
    if (lane < N) {
#pragma unroll
        for (int c = 0; c < N; ++c) w.u[lane * (N + 1) + c] = U[c];
    }
    wave_lds_sync();
    // t_c = sum_k U[k][c] rhs_k
    double tc = 0.0;
    if (lane < N) {
        for (int k = 0; k < N; ++k) {
            const double r = OBS ? (k < nz ? w.dt[k] : 0.0) : w.rhs[k];
            tc += w.u[k * (N + 1) + lane] * r;
        }
    }
    double e[9];
    if constexpr (OBS) {
        // B[a][j] = sqrt(r_j) sum_m dX[a][m] dY[q_j][m]
        double bj[9];
#pragma unroll
        for (int a = 0; a < 9; ++a) bj[a] = 0.0;
        if (lane < nz) {
            const double* row = p.dY + (size_t)w.q[lane] * M;
            for (int m = 0; m < M; ++m) {
                const double yv = row[m];
#pragma unroll
                for (int a = 0; a < 9; ++a) bj[a] += w.dx[a * 64 + m] * yv;
            }
            const double swj = w.sw[lane];
#pragma unroll
            for (int a = 0; a < 9; ++a) bj[a] *= swj;
        }
        if (lane < N) {
#pragma unroll
            for (int a = 0; a < 9; ++a) w.b[a * N + lane] = bj[a];
        }
        wave_lds_sync();
        // E = B U
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            double acc = 0.0;
            if (lane < N)
                for (int k = 0; k < N; ++k) acc += w.b[a * N + k] * w.u[k * (N + 1) + lane];
            e[a] = acc;
        }
    } else {
        // E = dX U
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            double acc = 0.0;
            if (lane < N)
                for (int k = 0; k < N; ++k) acc += w.dx[a * 64 + k] * w.u[k * (N + 1) + lane];
            e[a] = acc;
        }
    }
    // mean increment dX w_bar = sum_c E[a][c] psi_c t_c
    double dmean[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) dmean[a] = wave_sum(lane < N ? e[a] * psi * tc : 0.0);
    if (lane < N) {
#pragma unroll
        for (int a = 0; a < 9; ++a) w.e[a * N + lane] = e[a] * phi;
    }
    wave_lds_sync();

    double xa[9];
    if constexpr (OBS) {
        // C[a][j] = sum_c E'[a][c] U[j][c]  (lane j, own row of U)
        if (lane < N) {
#pragma unroll
            for (int a = 0; a < 9; ++a) {
                double acc = 0.0;
#pragma unroll
                for (int c = 0; c < N; ++c) acc += w.e[a * N + c] * U[c];
                w.b[a * N + lane] = acc;
            }
        }
        wave_lds_sync();
        double acc[9];
#pragma unroll
        for (int a = 0; a < 9; ++a) acc[a] = 0.0;
        if (mem) {
            for (int j = 0; j < nz; ++j) {
                const double z = w.sw[j] * p.dY[(size_t)w.q[j] * M + lane];
#pragma unroll
                for (int a = 0; a < 9; ++a) acc[a] += w.b[a * N + j] * z;
            }
        }
#pragma unroll
        for (int a = 0; a < 9; ++a) xa[a] = xbar[a] + p.sqrt_beta * dx[a] + dmean[a] + acc[a];
    } else {
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            double acc = 0.0;
#pragma unroll
            for (int c = 0; c < N; ++c) acc += w.e[a * N + c] * U[c];
            xa[a] = xbar[a] + dmean[a] + acc;
        }
    }
    if (mem) {
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            const int xs = wrap(x - cx_of(a), nx), ys = wrap(y - cy_of(a), ny);
            p.f[((size_t)lane * 9 + a) * plane + (size_t)ys * nx + xs] = xa[a];
        }
    }
}

// ---------------------------------------------------------------------------
// diagnostics: RMSE of the ensemble-mean velocity, spread, non-finite count,
// density range.  Deterministic two-pass reduction.
// ---------------------------------------------------------------------------
constexpr int kDiagBlock = 256;
constexpr int kDiagFields = 5;  // err2, spread2, nonfinite, rho_min, rho_max

__global__ __launch_bounds__(kDiagBlock) void diag_partial_kernel(
    const double* __restrict__ f, const double* __restrict__ truth_uv, int nx, int ny,
    int members, double* __restrict__ partial) {
    const int plane = nx * ny;
    double err2 = 0.0, spr2 = 0.0, bad = 0.0, rmin = INFINITY, rmax = -INFINITY;
    for (int i = blockIdx.x * kDiagBlock + threadIdx.x; i < plane; i += gridDim.x * kDiagBlock) {
        const int y = i / nx, x = i - y * nx;
        double su = 0.0, sv = 0.0, suu = 0.0;
        for (int m = 0; m < members; ++m) {
            double rho = 0.0, jx = 0.0, jy = 0.0;
#pragma unroll
            for (int a = 0; a < 9; ++a) {
                const int xs = wrap(x - cx_of(a), nx), ys = wrap(y - cy_of(a), ny);
                const double fa = f[((size_t)m * 9 + a) * plane + (size_t)ys * nx + xs];
                rho += fa;
                jx += cx_of(a) * fa;
                jy += cy_of(a) * fa;
            }
            const double u = jx / rho, v = jy / rho;
            if (!isfinite(rho) || !isfinite(u) || !isfinite(v)) bad += 1.0;
            rmin = fmin(rmin, rho);
            rmax = fmax(rmax, rho);
            su += u;
            sv += v;
            suu += u * u + v * v;
        }
        const double ub = su / members, vb = sv / members;
        if (truth_uv) {
            const double du = ub - truth_uv[i], dv = vb - truth_uv[plane + i];
            err2 += du * du + dv * dv;
        }
        if (members > 1) spr2 += (suu - members * (ub * ub + vb * vb)) / (members - 1);
    }
    __shared__ double red[kDiagFields][kDiagBlock];
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
        for (int k = 0; k < kDiagFields; ++k) partial[(size_t)blockIdx.x * kDiagFields + k] = red[k][0];
    }
}

__global__ void diag_final_kernel(const double* __restrict__ partial, int nblocks, int plane,
                                  double* __restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double err2 = 0.0, spr2 = 0.0, bad = 0.0, rmin = INFINITY, rmax = -INFINITY;
    for (int b = 0; b < nblocks; ++b) {
        err2 += partial[b * kDiagFields + 0];
        spr2 += partial[b * kDiagFields + 1];
        bad += partial[b * kDiagFields + 2];
        rmin = fmin(rmin, partial[b * kDiagFields + 3]);
        rmax = fmax(rmax, partial[b * kDiagFields + 4]);
    }
    out[0] = sqrt(err2 / plane);
    out[1] = sqrt(spr2 / plane);
    out[2] = bad;
    out[3] = rmin;
    out[4] = rmax;
    out[5] = 0.0;
    out[6] = 0.0;
    out[7] = 0.0;
}

__global__ void synth_obs_kernel(const double* __restrict__ y, const double* __restrict__ eps,
                                 const double* __restrict__ sigma, double* __restrict__ yo,
                                 int n) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) yo[q] = y[q] + sigma[q] * eps[q];
}

template <int N, bool OBS>
hipError_t launch_one(const AnalysisParams& p, hipStream_t s) {
    const int nz = p.nvar * p.lmax;
    const int per_wave = lds_doubles_per_wave(N, nz);
    const size_t bytes = (size_t)per_wave * sizeof(double);
    const int plane = p.nx * p.ny;
    analysis_kernel<N, OBS><<<plane, 64, bytes, s>>>(p, per_wave, 30);
    return hipGetLastError();
}

template <bool OBS>
hipError_t launch_sized(const AnalysisParams& p, int n, hipStream_t s) {
    switch (n) {
        case 8: return launch_one<8, OBS>(p, s);
        case 16: return launch_one<16, OBS>(p, s);
        case 24: return launch_one<24, OBS>(p, s);
        case 32: return launch_one<32, OBS>(p, s);
        case 48: return launch_one<48, OBS>(p, s);
        case 64: return launch_one<64, OBS>(p, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

int analysis_size_for(int n) {
    const int sizes[] = {8, 16, 24, 32, 48, 64};
    for (int v : sizes)
        if (n <= v) return v;
    return 0;
}

int analysis_lds_bytes(int n, int nz) { return lds_doubles_per_wave(n, nz) * (int)sizeof(double); }

hipError_t launch_observe(const double* f, const int* pts, int npts, int nvar, double* yf,
                          LbmDims d, hipStream_t s) {
    const int total = npts * d.members;
    observe_kernel<<<(total + 255) / 256, 256, 0, s>>>(f, pts, npts, nvar, yf, d.nx, d.ny,
                                                        d.members);
    return hipGetLastError();
}

hipError_t launch_obs_stats(const double* yf, const double* yo, int nobs, int members,
                            double* ybar, double* dY, double* dvec, double* K, hipStream_t s) {
    obs_stats_kernel<<<(nobs + 127) / 128, 128, 0, s>>>(yf, yo, nobs, members, ybar, dY, dvec);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !K) return e;
    const int total = nobs * nobs;
    obs_gram_kernel<<<(total + 255) / 256, 256, 0, s>>>(dY, nobs, members, K);
    return hipGetLastError();
}

hipError_t launch_local_table(const int* pts, int npts, double d_cut, int lmax, int nx, int ny,
                              int* loc_pt, double* loc_g, int* overflow, hipStream_t s) {
    const int plane = nx * ny;
    local_table_kernel<<<(plane + 255) / 256, 256, 0, s>>>(pts, npts, d_cut, lmax, nx, ny, loc_pt,
                                                            loc_g, overflow);
    return hipGetLastError();
}

hipError_t launch_analysis(const AnalysisParams& p, int route, int n, hipStream_t s) {
    return route == 2 ? launch_sized<true>(p, n, s) : launch_sized<false>(p, n, s);
}

hipError_t launch_diag(const double* f, const double* truth_uv, LbmDims d, double* partial,
                       int nblocks, double* out, hipStream_t s) {
    diag_partial_kernel<<<nblocks, kDiagBlock, 0, s>>>(f, truth_uv, d.nx, d.ny, d.members,
                                                       partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    diag_final_kernel<<<1, 64, 0, s>>>(partial, nblocks, d.nx * d.ny, out);
    return hipGetLastError();
}

hipError_t launch_synth_obs(const double* y, const double* eps, const double* sigma, double* yo,
                            int n, hipStream_t s) {
    synth_obs_kernel<<<(n + 255) / 256, 256, 0, s>>>(y, eps, sigma, yo, n);
    return hipGetLastError();
}

}  // namespace lbmletkf
