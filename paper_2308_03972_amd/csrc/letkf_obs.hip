// Observation-route LETKF analysis (Sec. 3.2.1, Sec. 3.2.2): for a node with
// l local observations the M x M ensemble-space matrix
// (M-1)/beta I + Z^T Z (Z = R_loc^-1/2 dY, l x M) is eigendecomposed through
// its l x l dual S = Z Z^T = U Lambda U^T: the dual's eigenpairs (lambda_i, u_i)
// give the eigenpairs ((M-1)/beta + lambda_i, Z^T u_i / sqrt(lambda_i)) and
// the eigenvalue (M-1)/beta on the orthogonal complement.  Hence
//   w_bar = Z^T U (a + Lambda)^-1 U^T d~,   a = (M-1)/beta,
//   dW    = sqrt(beta) I + Z^T G Z,  G = U phi(Lambda) U^T,
//   phi(l) = (sqrt((M-1)/(a+l)) - sqrt(beta)) / l = -sqrt(beta) / (a s (1+s)),
//   s = sqrt(1 + l/a)   (cancellation-free, finite at l = 0),
// and, with B = dX Z^T (9 x l) and h = U (a + Lambda)^-1 U^T d~,
//   x_m^a = x_bar + sqrt(beta) dX_m + B h + (B G) Z_m.
//
// Two kernels per group of nodes with the same eigenproblem size N (the
// smallest instantiated even size >= l):
//   analysis_eig_kernel<N>  64/N nodes per wavefront (a segment of N lanes per
//     node): local observations, S, the Jacobi eigensolver, and per node the
//     l x l matrix G and the vector h, written to a buffer;
//   analysis_apply_kernel   one node per wavefront, lane = member: x_bar, dX,
//     B, B G, B h and the update of the nine populations.
// Splitting keeps the register- and LDS-heavy eigensolver apart from the
// memory-bound state pass, so each runs at its own occupancy.
#include "common.h"
#include "device_util.h"

namespace lbmletkf {
namespace {
using namespace dev;

// ---------------------------------------------------------------------------
// eigen part: SEGS = 64 / N nodes per wavefront
// ---------------------------------------------------------------------------
// The Jacobi of the one-wavefront eigen kernels with skewed rows (P = 0 rounds
// by DPP, device_util.h) where their larger LDS rows keep the occupancy the
// registers allow; at N = 8, 12-16, 20 and 32 plain rows already fill, or
// nearly fill, the LDS at that occupancy and stay.
template <int N>
constexpr bool kSkewRows = N == 10 || N == 18 || (N >= 22 && N <= 30);

template <int N>
struct EigLayout {
    static_assert(N >= 8 && N % 2 == 0, "eigenproblem size must be even and >= 8");
    static constexpr int SEGS = 64 / N;
    static constexpr int RS = kSkewRows<N> ? SkewStride<N>::value : RowStride<N>::value;
    // Jacobi rows (also the convergence partial sums between sweeps), then U
    static constexpr int kRows = SEGS * N * RS > 128 ? SEGS * N * RS : 128;
    // (c, s) during Jacobi; psi t, phi, h after
    static constexpr int kCs = kSkewRows<N> ? skew_cs_doubles<N, SEGS>() : 2 * 64;
    static constexpr int kVec = kCs > 3 * 64 ? kCs : 3 * 64;
    static constexpr int kObs = 2 * SEGS * N + (SEGS * N + 1) / 2;  // sw, dt, q
    static constexpr int total = kRows + kVec + kObs;
};

// Local observation j of `node`: index q into the observation vector, weight
// sqrt(g / sigma^2) (R_loc^-1/2) and its innovation scaled by that weight.
__device__ __forceinline__ void local_obs(const AnalysisParams& p, int node, int j, int* q,
                                          double* w, double* d) {
    *q = 0;
    *w = 0.0;
    if (d) *d = 0.0;
    if (j >= p.nvar * p.lmax) return;
    const int slot = j / p.nvar, var = j - slot * p.nvar;
    const int k = p.loc_pt[(size_t)node * p.lmax + slot];
    if (k < 0) return;
    *q = k * p.nvar + var;
    *w = sqrt(p.loc_g[(size_t)node * p.lmax + slot] * p.rinv[var]);
    if (d) *d = *w * p.dvec[*q];
}

// One wavefront: the nodes nodes[item0 + seg] (seg < SEGS, item < end) of one problem.
template <int N>
__device__ __forceinline__ void eig_body(const AnalysisParams p, const int* nodes, int item0,
                                         int end, double* gout) {
    using L = EigLayout<N>;
    constexpr int SEGS = L::SEGS;
    constexpr int RS = L::RS;
    extern __shared__ double lds[];
    double* rows = lds;                              // [SEGS][N][RS]
    double* vec = rows + L::kRows;                   // [3][64]
    double* sw = vec + L::kVec;                      // [SEGS][N]
    double* dt = sw + SEGS * N;                      // [SEGS][N]
    int* qx = reinterpret_cast<int*>(dt + SEGS * N); // [SEGS][N]
    double2* cs = reinterpret_cast<double2*>(vec);   // Jacobi only
    double* pt = vec;                                // psi_c t_c
    double* phv = vec + 64;                          // phi_c

    const int lane = threadIdx.x;
    const int seg = lane / N;
    const int i = lane - seg * N;
    const bool active = seg < SEGS;
    const int sbase = active ? seg * N : 0;
    const int item = item0 + (active ? seg : 0);
    const bool valid = active && item < end;
    const int node = valid ? nodes[item] : 0;

    if (active) {
        int q = 0;
        double w = 0.0, d = 0.0;
        if (valid) local_obs(p, node, i, &q, &w, &d);
        qx[lane] = q;
        sw[lane] = w;
        dt[lane] = d;
    }
    wave_lds_sync();
    // S = Z Z^T = diag(sw) K diag(sw) on the local observations
    double S[N], U[N];
    {
        const double wi = active ? sw[lane] : 0.0;
        const double* Krow = p.K + (size_t)(active ? qx[lane] : 0) * p.nobs;
        // unconditional loads (an unused entry has index 0), so that all N are
        // in flight together; the weights select afterwards
#pragma unroll
        for (int k = 0; k < N; ++k) S[k] = Krow[qx[sbase + k]];
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const double wk = sw[sbase + k];
            S[k] = (wi != 0.0 && wk != 0.0) ? wi * wk * S[k] : 0.0;
            U[k] = (k == i && active) ? 1.0 : 0.0;
        }
    }
    int sweeps;
    if constexpr (kSkewRows<N>) sweeps = jacobi_eig_skew<N, SEGS>(S, U, rows, cs, lane, p.max_sweeps);
    else sweeps = jacobi_eig<N, SEGS>(S, U, rows, cs, rows, lane, p.max_sweeps);
    if (sweeps > p.max_sweeps && lane == 0) atomicAdd(p.eig_fail, 1);

    // eigenvalue functions, U to LDS, t = U^T d~, h = U psi t, G = U phi U^T
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
    phv[lane] = active ? phi : 0.0;
    wave_lds_sync();
    {
        double t = 0.0;
        if (active)
            for (int k = 0; k < N; ++k) t += rows[(size_t)(sbase + k) * RS + i] * dt[sbase + k];
        pt[lane] = active ? psi * t : 0.0;
    }
    wave_lds_sync();
    double h = 0.0;
#pragma unroll
    for (int c = 0; c < N; ++c) h += U[c] * pt[sbase + c];
    // row i of U phi, in place
#pragma unroll
    for (int c = 0; c < N; ++c) U[c] *= phv[sbase + c];
    if (valid) {
        // lane i computes G_ij = sum_c U_ic phi_c U_jc and stores it at (j, i):
        // consecutive lanes write consecutive addresses
        double* out = gout + (size_t)item * (N * N + N);
#pragma unroll 1
        for (int j = 0; j < N; ++j) {
            const double2* rj = reinterpret_cast<const double2*>(rows + (size_t)(sbase + j) * RS);
            double g = 0.0;
#pragma unroll
            for (int c = 0; c < N / 2; ++c) {
                const double2 r = rj[c];
                g += U[2 * c] * r.x + U[2 * c + 1] * r.y;
            }
            out[(size_t)j * N + i] = g;
        }
        out[(size_t)N * N + i] = h;
    }
}

// ---------------------------------------------------------------------------
// eigen part for N > 32: one node per block of two wavefronts, every row split
// between them -- thread (h, i) holds columns [h H, (h + 1) H) of row i of S and
// of U (H = N / 2), N doubles per lane instead of 2 N, so two blocks fit per SIMD
// pair instead of one wavefront.  Same rounds as the one-wavefront solver: the
// half rows are published to LDS, half 0 derives each pair's (c, s) from the
// published 2 x 2 blocks, every thread mixes its half row with the partner's
// published half row and rotates the column pairs inside its half; the one
// column pair that straddles the halves (H - 1, H), paired when P = 1, is
// finished after trading its two entries of S and U through LDS.
// ---------------------------------------------------------------------------
template <int N>
struct SplitLayout {
    static_assert(N > 32 && N <= 64 && N % 4 == 0, "split rows need 32 < N <= 64, N / 2 even");
    static constexpr int H = N / 2;
    static constexpr int RS = RowStride<N>::value;
    static constexpr int kThreads = 2 * kWave;
    static constexpr int kRows = 2 * N * RS;       // published S, two buffers by round parity;
                                                   // afterwards U and the G partial sums
    static constexpr int kCs = 2 * 2 * N;          // (c, s) per row, one list per wavefront
    static constexpr int kRed = 2 * kThreads;      // convergence partial sums
    static constexpr int kBx = 4 * N;              // straddling column of S and U, per half
    static constexpr int kVec = 3 * N;             // eigenvalues, psi t, phi
    static constexpr int kObs = 2 * N + (N + 1) / 2;  // sw, dt, q
    static constexpr int total = kRows + kCs + kRed + kBx + kVec + kObs;
};

// One round: publish the half rows into buffer `rows` (the two buffers
// alternate, so the previous round's readers need no barrier), then every
// thread derives its own pair's (c, s) from the published 2 x 2 block (both
// halves of a row get identical values) and shares it within its wavefront,
// whose column range needs only its own rows' rotations.
template <int N, int P>
__device__ __forceinline__ void split_round(double (&S)[N / 2], double (&U)[N / 2], double* rows,
                                            double2* csw, double* bx, int i, int hh, bool active) {
    constexpr int H = N / 2;
    constexpr int RS = RowStride<N>::value;
    const int c0 = hh * H;
    if (active) {
        double2* my = reinterpret_cast<double2*>(rows + (size_t)i * RS + c0);
#pragma unroll
        for (int k = 0; k < H / 2; ++k) my[k] = make_double2(S[2 * k], S[2 * k + 1]);
    }
    __syncthreads();
    const bool first = ((i - P) & 1) == 0;
    const int pi = first ? i + 1 : i - 1;
    const bool paired = active && pi >= 0 && pi < N;
    // a thread without a partner reads the first pair's block and discards it
    const int p = paired ? (first ? i : pi) : 0;
    double c, s;
    jacobi_rotation(rows[(size_t)p * RS + p], rows[(size_t)(p + 1) * RS + p + 1],
                    rows[(size_t)p * RS + p + 1], paired, &c, &s);
    if (active) csw[i] = make_double2(c, s);
    wave_lds_sync();
    const double sg = first ? s : -s;
    // row mix from the partner's published half row (own row, c = 1, s = 0 for
    // a row without a partner), then the column pairs inside this half
    const int src = paired ? pi : (active ? i : 0);
    const double2* pr = reinterpret_cast<const double2*>(rows + (size_t)src * RS + c0);
#pragma unroll
    for (int k = 0; k < H / 2; ++k) {
        const double2 v = pr[k];
        S[2 * k] = c * v.x + sg * S[2 * k];
        S[2 * k + 1] = c * v.y + sg * S[2 * k + 1];
        const int r = 2 * k - P;
        if (r >= 0) {
            const double2 q = csw[c0 + r];
            const double a0 = S[r], a1 = S[r + 1];
            S[r] = q.y * a0 + q.x * a1;
            S[r + 1] = q.x * a0 - q.y * a1;
            const double u0 = U[r], u1 = U[r + 1];
            U[r] = q.y * u0 + q.x * u1;
            U[r + 1] = q.x * u0 - q.y * u1;
        }
    }
    if (P == 1) {
        // the pair (H - 1, H): half 0 holds entry H - 1 (its last), half 1 entry H (its first)
        if (active) {
            bx[(size_t)(2 * hh) * N + i] = hh == 0 ? S[H - 1] : S[0];
            bx[(size_t)(2 * hh + 1) * N + i] = hh == 0 ? U[H - 1] : U[0];
        }
        __syncthreads();
        if (active) {
            const double2 q = csw[H - 1];
            const double so = bx[(size_t)(2 * (1 - hh)) * N + i];
            const double uo = bx[(size_t)(2 * (1 - hh) + 1) * N + i];
            if (hh == 0) {
                S[H - 1] = q.y * S[H - 1] + q.x * so;
                U[H - 1] = q.y * U[H - 1] + q.x * uo;
            } else {
                S[0] = q.x * so - q.y * S[0];
                U[0] = q.x * uo - q.y * U[0];
            }
        }
    }
#pragma unroll
    for (int r = 0; r < H; ++r) asm volatile("" : "+v"(U[r]), "+v"(S[r]));
}

// One block of two wavefronts: node nodes[item] (item < end) of one problem.
template <int N>
__device__ __forceinline__ void eig_body_split(const AnalysisParams p, const int* nodes, int item,
                                               int end, double* gout) {
    using L = SplitLayout<N>;
    constexpr int H = L::H;
    constexpr int RS = L::RS;
    extern __shared__ double lds[];
    double* rows = lds;                                   // [2][N][RS]
    double* xg = rows + N * RS;                           // second buffer, after the sweeps
    double2* cs = reinterpret_cast<double2*>(rows + L::kRows);  // [2 halves][N]
    double* red = rows + L::kRows + L::kCs;               // [2 * 128]
    double* bx = red + L::kRed;                           // [2 halves][S, U][N]
    double* lam = bx + L::kBx;                            // [N]
    double* pt = lam + N;                                 // [N]
    double* phv = pt + N;                                 // [N]
    double* sw = phv + N;                                 // [N]
    double* dt = sw + N;                                  // [N]
    int* qx = reinterpret_cast<int*>(dt + N);             // [N]

    const int t = threadIdx.x;
    const int hh = t / kWave;
    const int i = t - hh * kWave;
    const bool active = i < N;
    const int c0 = hh * H;
    const bool valid = item < end;
    const int node = valid ? nodes[item] : 0;

    if (hh == 0 && active) {
        int q = 0;
        double w = 0.0, d = 0.0;
        if (valid) local_obs(p, node, i, &q, &w, &d);
        qx[i] = q;
        sw[i] = w;
        dt[i] = d;
    }
    __syncthreads();
    // this thread's half of row i of S = diag(sw) K diag(sw), and of U = I
    double S[H], U[H];
    {
        const double wi = active ? sw[i] : 0.0;
        const double* Krow = p.K + (size_t)(active ? qx[i] : 0) * p.nobs;
        // unconditional loads (an unused entry has index 0), all in flight together
#pragma unroll
        for (int k = 0; k < H; ++k) S[k] = Krow[qx[c0 + k]];
#pragma unroll
        for (int k = 0; k < H; ++k) {
            const double wk = sw[c0 + k];
            S[k] = (wi != 0.0 && wk != 0.0) ? wi * wk * S[k] : 0.0;
            U[k] = (active && c0 + k == i) ? 1.0 : 0.0;
        }
    }
    // sweeps until the off-diagonal Frobenius norm is below 1e-13 of the
    // diagonal's; every thread sums the same partials in the same order
    int sweeps = 0;
    for (;; ++sweeps) {
        double off = 0.0, dg = 0.0;
#pragma unroll
        for (int k = 0; k < H; ++k) {
            const double v2 = S[k] * S[k];
            if (c0 + k == i) dg += v2;
            else off += v2;
        }
        __syncthreads();
        red[2 * t] = active ? off : 0.0;
        red[2 * t + 1] = active ? dg : 0.0;
        __syncthreads();
        double so = 0.0, sd = 0.0;
        for (int k = 0; k < L::kThreads; ++k) {
            so += red[2 * k];
            sd += red[2 * k + 1];
        }
        if (so <= 1e-26 * sd) break;
        if (sweeps >= p.max_sweeps) {
            sweeps = p.max_sweeps + 1;
            break;
        }
        double2* mycs = cs + hh * N;
#pragma unroll 1
        for (int rr = 0; rr < N / 2; ++rr) {
            split_round<N, 0>(S, U, rows, mycs, bx, i, hh, active);
            split_round<N, 1>(S, U, rows + N * RS, mycs, bx, i, hh, active);
        }
    }
    if (sweeps > p.max_sweeps && t == 0) atomicAdd(p.eig_fail, 1);

    // eigenvalues (the diagonal entry of row i sits in half i / H), U to LDS
    __syncthreads();
    if (active && i / H == hh) lam[i] = extract_lane_entry<H>(S, i - c0);
    if (active) {
        double2* my = reinterpret_cast<double2*>(rows + (size_t)i * RS + c0);
#pragma unroll
        for (int k = 0; k < H / 2; ++k) my[k] = make_double2(U[2 * k], U[2 * k + 1]);
    }
    __syncthreads();
    // phi_c, and psi_c t_c with t = U^T d~ (thread (0, c) for column c)
    if (hh == 0 && active) {
        const double lm = lam[i];
        const double sq = sqrt(1.0 + lm / p.a);
        const double psi = 1.0 / (p.a + lm);
        phv[i] = -p.sqrt_beta / (p.a * sq * (1.0 + sq));
        double tt = 0.0;
        for (int k = 0; k < N; ++k) tt += rows[(size_t)k * RS + i] * dt[k];
        pt[i] = psi * tt;
    }
    __syncthreads();
    // G_ij = sum_c U_ic phi_c U_jc: each half sums its own columns c; a thread
    // hands the partial sums for the other half's outputs j over through LDS
#pragma unroll
    for (int k = 0; k < H; ++k) U[k] *= phv[c0 + k];
    const int oc0 = (1 - hh) * H;
    if (active) {
#pragma unroll 1
        for (int j = oc0; j < oc0 + H; ++j) {
            const double2* rj = reinterpret_cast<const double2*>(rows + (size_t)j * RS + c0);
            double g = 0.0;
#pragma unroll
            for (int k = 0; k < H / 2; ++k) {
                const double2 r = rj[k];
                g += U[2 * k] * r.x + U[2 * k + 1] * r.y;
            }
            xg[(size_t)i * RS + j] = g;
        }
    }
    __syncthreads();
    if (active && valid) {
        double* out = gout + (size_t)item * (N * N + N);
#pragma unroll 1
        for (int j = c0; j < c0 + H; ++j) {
            const double2* rj = reinterpret_cast<const double2*>(rows + (size_t)j * RS + c0);
            double g = 0.0;
#pragma unroll
            for (int k = 0; k < H / 2; ++k) {
                const double2 r = rj[k];
                g += U[2 * k] * r.x + U[2 * k + 1] * r.y;
            }
            out[(size_t)j * N + i] = g + xg[(size_t)i * RS + j];
        }
        if (hh == 0) {
            double hs = 0.0;
            for (int c = 0; c < N; ++c) hs += rows[(size_t)i * RS + c] * pt[c];
            out[(size_t)N * N + i] = hs;
        }
    }
}

// Split rows above N = 32.  At N = 32 itself one wavefront holding two nodes
// with whole rows beats one node with half rows in a wavefront (measured 103
// against 134 ns per node at 64 members).  The eigensolver fits in 128 VGPRs
// (four wavefronts per SIMD) up to N = 16 and in 168 (three) up to N = 22
// without spilling; N = 24 with skewed rows would spill 40 bytes per lane at
// three and keeps two.  Four wavefronts per SIMD at N = 18-22 were measured no
// faster (with plain rows): the rounds are held by the LDS traffic of the row
// exchange and the rotation broadcast and by their latency, not by occupancy.
template <int N>
constexpr bool kSplitRows = N > 32;

template <int N>
constexpr int eig_threads() { return kSplitRows<N> ? 2 * kWave : kWave; }

template <int N>
constexpr int eig_waves() { return N <= 16 ? 4 : (N <= 22 ? 3 : 1); }

template <int N>
constexpr int eig_lds_doubles() {
    if constexpr (kSplitRows<N>) return SplitLayout<N>::total;
    else return EigLayout<N>::total;
}

template <int N>
__global__ __launch_bounds__(eig_threads<N>()) __attribute__((amdgpu_waves_per_eu(eig_waves<N>())))
void analysis_eig_kernel(AnalysisParams p, const int* nodes, int count, double* gout) {
    if constexpr (kSplitRows<N>)
        eig_body_split<N>(p, nodes, xcd_remap(blockIdx.x, gridDim.x), count, gout);
    else
        eig_body<N>(p, nodes, xcd_remap(blockIdx.x, gridDim.x) * EigLayout<N>::SEGS, count, gout);
}

// Batched form: wavefront w takes waves[w] = (problem, first item, end of the
// problem's items); the items of all problems share one node list and one G buffer.
template <int N>
__global__ __launch_bounds__(eig_threads<N>()) __attribute__((amdgpu_waves_per_eu(eig_waves<N>())))
void analysis_eig_batch_kernel(const AnalysisParams* P, const int4* waves, int nwaves,
                               const int* nodes, double* gout) {
    const int w = xcd_remap(blockIdx.x, gridDim.x);
    if (w >= nwaves) return;
    const int4 d = waves[w];
    const AnalysisParams p = P[d.x];
    if constexpr (kSplitRows<N>) eig_body_split<N>(p, nodes, d.y, d.z, gout);
    else eig_body<N>(p, nodes, d.y, d.z, gout);
}

// Dynamic LDS beyond 64 KiB needs the kernel's permission (set once per kernel).
template <typename K>
hipError_t allow_lds(K kernel, size_t bytes, bool* done) {
    if (bytes <= 65536 || *done) return hipSuccess;
    hipError_t e = hipFuncSetAttribute((const void*)kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess) *done = true;
    return e;
}

// ---------------------------------------------------------------------------
// apply part: one node per wavefront, lane = member
// ---------------------------------------------------------------------------
__host__ __device__ inline int apply_lds_doubles(int n) {
    // G and h, dX [9][64], B [9][n], C [n][10], sw [n], mean increment [9],
    // x_bar [9], q [n]
    return n * n + n + 9 * 64 + 9 * n + 10 * n + n + 9 + 9 + (n + 1) / 2;
}

// One wavefront: node nodes[item] of one problem, lane = member.
template <int N, typename T>
__device__ __forceinline__ void apply_body(const AnalysisParams& p, const int* nodes, int item,
                                           const double* __restrict__ gin) {
    constexpr int n = N;
    constexpr int groups = kWave / N;                  // member groups in B
    constexpr int kChunk = (kWave + groups - 1) / groups;
    T* __restrict__ fs = reinterpret_cast<T*>(p.f);
    extern __shared__ double lds[];
    double* Gs = lds;                                  // [n][n] as stored: (k, j) = G_jk
    double* hs = Gs + n * n;                           // [n]
    double* dxs = hs + n;                              // [9][64]
    double* Bs = dxs + 9 * 64;                         // [9][n]
    double* Cs = Bs + 9 * n;                           // [n][10]
    double* sw = Cs + 10 * n;                          // [n]
    double* dmv = sw + n;                              // [9]
    double* xbv = dmv + 9;                             // [9]
    int* qx = reinterpret_cast<int*>(xbv + 9);         // [n]

    const int lane = threadIdx.x;
    const int node = nodes[item];
    const int nx = p.nx, ny = p.ny, M = p.members;
    const bool mem = lane < M;
    const int x = node % nx, y = node / nx;

    // independent loads first, in one block so that they are all in flight
    // before the first use: the nine populations, G and h (the last pass
    // clamps its index), this lane's local observation
    constexpr int kGn = n * n + n;
    constexpr int kGp = (kGn + kWave - 1) / kWave;
    double dx[9];
    const int ml = mem ? lane : 0;  // a lane past the ensemble reads member 0 and discards it
#pragma unroll
    for (int a = 0; a < 9; ++a)
        dx[a] = PopIO<T>::load(fs + slot(src_node(x, y, a, nx, ny), a, ml, M), a);
#pragma unroll
    for (int a = 0; a < 9; ++a) dx[a] = mem ? dx[a] : 0.0;
    const double* g = gin + (size_t)item * kGn;
    double gv[kGp];
#pragma unroll
    for (int u = 0; u < kGp; ++u) gv[u] = g[min(lane + u * kWave, kGn - 1)];
    int qj = 0;
    double wj = 0.0;
    if (lane < n) local_obs(p, node, lane, &qj, &wj, nullptr);
    if (p.diag_node)
        node_diag_record(dx, mem, M, node, nx * ny, p.truth_uv,
                         p.diag_node + (size_t)node * kDiagFieldCount);
#pragma unroll
    for (int u = 0; u < kGp; ++u)
        if (lane + u * kWave < kGn) Gs[lane + u * kWave] = gv[u];
    if (lane < n) {
        qx[lane] = qj;
        sw[lane] = wj;
    }
    wave_lds_sync();
    // x_bar and dX of the nine populations
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const double xbar = wave_sum(dx[a]) / M;
        dx[a] = mem ? dx[a] - xbar : 0.0;
        dxs[a * 64 + lane] = dx[a];
        if (lane == 0) xbv[a] = xbar;
    }
    wave_lds_sync();
    // B[a][j] = w_j sum_m dX_a(m) dY[q_j][m]: lane (group, j) sums a member
    // range (its dY values loaded together first), the groups are combined in a
    // fixed order
    const int gi = lane / n, j = lane - gi * n;
    const bool gact = gi < groups;
    double b[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) b[a] = 0.0;
    if (gact && sw[j] != 0.0) {
        const int mchunk = (M + groups - 1) / groups;
        const int m0 = gi * mchunk;
        const int m1 = min(M, m0 + mchunk);
        const double* yrow = p.dY + (size_t)qx[j] * M;
        double yv[kChunk];
#pragma unroll
        for (int t = 0; t < kChunk; ++t) yv[t] = m0 + t < m1 ? yrow[m0 + t] : 0.0;
#pragma unroll
        for (int t = 0; t < kChunk; ++t) {
            const int m = m0 + t < m1 ? m0 + t : m0;
#pragma unroll
            for (int a = 0; a < 9; ++a) b[a] += dxs[a * 64 + m] * yv[t];
        }
    }
    for (int gg = 1; gg < groups; ++gg) {
        const int src = gact ? j + gg * n : lane;
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            const double v = __shfl(b[a], src, kWave);
            b[a] += (gi == 0) ? v : 0.0;
        }
    }
    if (lane < n) {
        const double wj = sw[lane];
#pragma unroll
        for (int a = 0; a < 9; ++a) Bs[a * n + lane] = b[a] * wj;
    }
    wave_lds_sync();
    // C = B G ([j][a]) and the mean increment B h
    for (int jj = lane; jj < n; jj += kWave) {
        double c[9];
#pragma unroll
        for (int a = 0; a < 9; ++a) c[a] = 0.0;
        for (int k = 0; k < n; ++k) {
            const double gkj = Gs[k * n + jj];
#pragma unroll
            for (int a = 0; a < 9; ++a) c[a] += Bs[a * n + k] * gkj;
        }
#pragma unroll
        for (int a = 0; a < 9; ++a) Cs[jj * 10 + a] = c[a];
        Cs[jj * 10 + 9] = 0.0;
    }
    if (lane < 9) {
        double d = 0.0;
        for (int k = 0; k < n; ++k) d += Bs[lane * n + k] * hs[k];
        dmv[lane] = d;
    }
    wave_lds_sync();
    double xa[9];  // the analysis as stored (diagnostics)
#pragma unroll
    for (int a = 0; a < 9; ++a) xa[a] = 0.0;
    if (mem) {
        // this member's l observation perturbations: unconditional loads (an
        // unused entry has index 0) so that all N are in flight together
        double z[N];
#pragma unroll
        for (int jj = 0; jj < N; ++jj) z[jj] = p.dY[(size_t)qx[jj] * M + lane];
#pragma unroll
        for (int jj = 0; jj < N; ++jj) {
            const double wj = sw[jj];
            z[jj] = wj != 0.0 ? wj * z[jj] : 0.0;
        }
        double acc[9];
#pragma unroll
        for (int a = 0; a < 9; ++a) acc[a] = 0.0;
#pragma unroll
        for (int jj = 0; jj < N; ++jj) {
            const double2* c2 = reinterpret_cast<const double2*>(Cs + jj * 10);
#pragma unroll
            for (int hh = 0; hh < 5; ++hh) {
                const double2 cv = c2[hh];
                acc[2 * hh] += cv.x * z[jj];
                if (2 * hh + 1 < 9) acc[2 * hh + 1] += cv.y * z[jj];
            }
            if (jj % 4 == 3) __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            const double v = xbv[a] + p.sqrt_beta * dx[a] + dmv[a] + acc[a];
            PopIO<T>::store(fs + slot(src_node(x, y, a, nx, ny), a, lane, M), a, v);
            xa[a] = PopIO<T>::round(v, a);
        }
    }
    if (p.diag_node)
        node_diag_record(xa, mem, M, node, nx * ny, p.truth_uv,
                         p.diag_node + ((size_t)nx * ny + node) * kDiagFieldCount);
}

// ---------------------------------------------------------------------------
// apply part of the precision form (FP32 storage): the two ensemble-space
// contractions per node, B = dX Z^T (9 x n, inner dimension the members) and
// the transform dX_inc = C^T Z (9 x M, inner dimension n, C = B G), on the
// BF16 matrix cores with FP32 accumulation.  Each FP32 operand x is split into
// x_hi = bf16(x) and x_lo = bf16(x - x_hi); a product is taken as
// hi*hi + hi*lo + lo*hi (the lo*lo term and the roundings leave ~2^-16
// relative), three v_mfma_f32_16x16x32_bf16 per tile.  Operand layout (per
// wavefront, lane l, element t < 8): A[l % 16][8 (l / 16) + t],
// B[8 (l / 16) + t][l % 16]; result register r of lane l holds
// D[4 (l / 16) + r][l % 16] (measured on gfx950).  Rows of A are the nine
// populations (padded to 16); everything else is as in apply_body.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void split_bf16(const float (&x)[8], bf16x8& hi, bf16x8& lo) {
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const __bf16 h = (__bf16)x[t];
        hi[t] = h;
        lo[t] = (__bf16)(x[t] - (float)h);
    }
}

__device__ __forceinline__ f32x4 mfma_bf16x3(const float (&a)[8], const float (&b)[8], f32x4 acc) {
    bf16x8 ah, al, bh, bl;
    split_bf16(a, ah, al);
    split_bf16(b, bh, bl);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc, 0, 0, 0);
}

template <int N>
__device__ __forceinline__ void apply_body_mfma(const AnalysisParams& p, const int* nodes, int item,
                                                const double* __restrict__ gin) {
    constexpr int n = N;
    constexpr int NT = (n + 15) / 16;  // column tiles of B
    static_assert(n <= 32, "one 32-deep step of the transform");
    float* __restrict__ fs = reinterpret_cast<float*>(p.f);
    extern __shared__ double lds[];
    double* Gs = lds;                                  // [n][n] as stored: (k, j) = G_jk
    double* hs = Gs + n * n;                           // [n]
    double* dxs = hs + n;                              // [9][64]
    double* Bs = dxs + 9 * 64;                         // [9][n]
    double* Cs = Bs + 9 * n;                           // [n][10]
    double* sw = Cs + 10 * n;                          // [n]
    double* dmv = sw + n;                              // [9]
    double* xbv = dmv + 9;                             // [9]
    int* qx = reinterpret_cast<int*>(xbv + 9);         // [n]
    // the transform's result [9][64] (FP32) reuses dX's region, which the
    // contraction B = dX Z^T has finished reading before the transform
    float* outs = reinterpret_cast<float*>(dxs);

    const int lane = threadIdx.x;
    const int node = nodes[item];
    const int nx = p.nx, ny = p.ny, M = p.members;
    const bool mem = lane < M;
    const int x = node % nx, y = node / nx;
    const int r16 = lane & 15, grp = lane >> 4;

    constexpr int kGn = n * n + n;
    constexpr int kGp = (kGn + kWave - 1) / kWave;
    double dx[9];
    const int ml = mem ? lane : 0;
#pragma unroll
    for (int a = 0; a < 9; ++a)
        dx[a] = PopIO<float>::load(fs + slot(src_node(x, y, a, nx, ny), a, ml, M), a);
#pragma unroll
    for (int a = 0; a < 9; ++a) dx[a] = mem ? dx[a] : 0.0;
    const double* g = gin + (size_t)item * kGn;
    double gv[kGp];
#pragma unroll
    for (int u = 0; u < kGp; ++u) gv[u] = g[min(lane + u * kWave, kGn - 1)];
    int qj = 0;
    double wj = 0.0;
    if (lane < n) local_obs(p, node, lane, &qj, &wj, nullptr);
    if (p.diag_node)
        node_diag_record(dx, mem, M, node, nx * ny, p.truth_uv,
                         p.diag_node + (size_t)node * kDiagFieldCount);
#pragma unroll
    for (int u = 0; u < kGp; ++u)
        if (lane + u * kWave < kGn) Gs[lane + u * kWave] = gv[u];
    if (lane < n) {
        qx[lane] = qj;
        sw[lane] = wj;
    }
    wave_lds_sync();
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const double xbar = wave_sum(dx[a]) / M;
        dx[a] = mem ? dx[a] - xbar : 0.0;
        dxs[a * 64 + lane] = dx[a];
        if (lane == 0) xbv[a] = xbar;
    }
    wave_lds_sync();
    // B = dX Z^T: A = dX (row a = l % 16, members 32 ks + 8 grp + t), B = Z^T
    // (members, column j = 16 tile + l % 16), two 32-member steps
    {
        f32x4 acc[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            const int m0 = 32 * ks + 8 * grp;
            float av[8];
#pragma unroll
            for (int t = 0; t < 8; ++t)
                av[t] = r16 < 9 ? (float)dxs[r16 * 64 + m0 + t] : 0.0f;
#pragma unroll
            for (int tile = 0; tile < NT; ++tile) {
                const int j = 16 * tile + r16;
                const bool jin = j < n;
                const double w = jin ? sw[j] : 0.0;
                const double* yrow = p.dY + (size_t)(jin ? qx[j] : 0) * M;
                float bv[8];
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    const int m = m0 + t;
                    const double yv = yrow[m < M ? m : 0];   // unconditional, selected below
                    bv[t] = (jin && m < M) ? (float)(w * yv) : 0.0f;
                }
                acc[tile] = mfma_bf16x3(av, bv, acc[tile]);
            }
        }
#pragma unroll
        for (int tile = 0; tile < NT; ++tile)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int a = 4 * grp + r, j = 16 * tile + r16;
                if (a < 9 && j < n) Bs[a * n + j] = (double)acc[tile][r];
            }
    }
    wave_lds_sync();
    // C = B G ([j][a]) and the mean increment B h (FP64 vector units)
    for (int jj = lane; jj < n; jj += kWave) {
        double c[9];
#pragma unroll
        for (int a = 0; a < 9; ++a) c[a] = 0.0;
        for (int k = 0; k < n; ++k) {
            const double gkj = Gs[k * n + jj];
#pragma unroll
            for (int a = 0; a < 9; ++a) c[a] += Bs[a * n + k] * gkj;
        }
#pragma unroll
        for (int a = 0; a < 9; ++a) Cs[jj * 10 + a] = c[a];
        Cs[jj * 10 + 9] = 0.0;
    }
    if (lane < 9) {
        double d = 0.0;
        for (int k = 0; k < n; ++k) d += Bs[lane * n + k] * hs[k];
        dmv[lane] = d;
    }
    wave_lds_sync();
    // transform: A = C^T (row a = l % 16, observations 8 grp + t), B = Z
    // (observations, member 16 tile + l % 16), four member tiles
    f32x4 tr[4];
    {
        float av[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int j = 8 * grp + t;
            av[t] = (r16 < 9 && j < n) ? (float)Cs[j * 10 + r16] : 0.0f;
        }
#pragma unroll
        for (int tile = 0; tile < 4; ++tile) {
            const int m = 16 * tile + r16;
            const int mm = m < M ? m : 0;
            float bv[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int j = 8 * grp + t;
                const bool jin = j < n;
                const double yv = p.dY[(size_t)qx[jin ? j : 0] * M + mm];
                bv[t] = (jin && m < M) ? (float)(sw[j] * yv) : 0.0f;
            }
            tr[tile] = mfma_bf16x3(av, bv, f32x4{0.0f, 0.0f, 0.0f, 0.0f});
        }
    }
    wave_lds_sync();
#pragma unroll
    for (int tile = 0; tile < 4; ++tile)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int a = 4 * grp + r;
            if (a < 9) outs[a * 64 + 16 * tile + r16] = tr[tile][r];
        }
    wave_lds_sync();
    double xa[9];  // the analysis as stored (diagnostics)
#pragma unroll
    for (int a = 0; a < 9; ++a) xa[a] = 0.0;
    if (mem) {
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            const double v = xbv[a] + p.sqrt_beta * dx[a] + dmv[a] + (double)outs[a * 64 + lane];
            PopIO<float>::store(fs + slot(src_node(x, y, a, nx, ny), a, lane, M), a, v);
            xa[a] = PopIO<float>::round(v, a);
        }
    }
    if (p.diag_node)
        node_diag_record(xa, mem, M, node, nx * ny, p.truth_uv,
                         p.diag_node + ((size_t)nx * ny + node) * kDiagFieldCount);
}

// The apply body of a node: with MF (FP32 storage, n <= 32) the matrix-core
// contractions, else the FP64 vector path.
template <int N>
constexpr bool kMfmaApply = N <= 32;

template <int N, typename T, bool MF>
__device__ __forceinline__ void apply_node(const AnalysisParams& p, const int* nodes, int item,
                                           const double* __restrict__ gin) {
    if constexpr (MF && sizeof(T) == 4 && kMfmaApply<N>) apply_body_mfma<N>(p, nodes, item, gin);
    else apply_body<N, T>(p, nodes, item, gin);
}

template <int N, typename T, bool MF>
__global__ __launch_bounds__(64) void analysis_apply_kernel(AnalysisParams p, const int* nodes,
                                                            int count,
                                                            const double* __restrict__ gin) {
    const int item = xcd_remap(blockIdx.x, gridDim.x);
    if (item >= count) return;  // uniform over the wavefront
    apply_node<N, T, MF>(p, nodes, item, gin);
}

// Batched form: wavefront w takes waves[w] = (problem, item).
template <int N, typename T, bool MF>
__global__ __launch_bounds__(64) void analysis_apply_batch_kernel(const AnalysisParams* P,
                                                                  const int2* waves, int nwaves,
                                                                  const int* nodes,
                                                                  const double* __restrict__ gin) {
    const int w = xcd_remap(blockIdx.x, gridDim.x);
    if (w >= nwaves) return;
    const int2 d = waves[w];
    const AnalysisParams p = P[d.x];
    apply_node<N, T, MF>(p, nodes, d.y, gin);
}

// Work-queue form of the batched kernels: a persistent grid whose blocks take
// entries of the group's wave list from queues in device memory until they are
// exhausted.  The list is cut into eight contiguous ranges, one per XCD (block
// b runs on XCD b mod 8), each with its own counter that a block advances by
// kQueueChunk entries with one lane's vector atomic add: one counter for the
// whole device would serialise every block's add across the XCDs.  Every block
// leaves once its counter has passed the end of its range; each entry is
// processed exactly as in the one-launch-per-wave form.
constexpr int kQueueChunk = 4;

__device__ __forceinline__ int queue_take(int* counters, int* next, int lo) {
    __syncthreads();  // the previous entries' LDS use ends before `next` is rewritten
    if (threadIdx.x == 0) *next = lo + atomicAdd(counters + blockIdx.x % 8, kQueueChunk);
    __syncthreads();
    return *next;
}

template <int N>
__global__ __launch_bounds__(eig_threads<N>()) __attribute__((amdgpu_waves_per_eu(eig_waves<N>())))
void analysis_eig_queue_kernel(const AnalysisParams* P, const int4* waves, int nwaves,
                               const int* nodes, double* gout, int* counters) {
    __shared__ int next;
    const int per = (nwaves + 7) / 8;
    const int lo = (int)(blockIdx.x % 8) * per;
    const int hi = min(nwaves, lo + per);
    for (;;) {
        const int w0 = queue_take(counters, &next, lo);
        if (w0 >= hi) return;  // uniform over the block
        const int w1 = min(hi, w0 + kQueueChunk);
        for (int w = w0; w < w1; ++w) {
            if (w > w0) __syncthreads();
            const int4 d = waves[w];
            const AnalysisParams p = P[d.x];
            if constexpr (kSplitRows<N>) eig_body_split<N>(p, nodes, d.y, d.z, gout);
            else eig_body<N>(p, nodes, d.y, d.z, gout);
        }
    }
}

template <int N, typename T, bool MF>
__global__ __launch_bounds__(64) void analysis_apply_queue_kernel(const AnalysisParams* P,
                                                                  const int2* waves, int nwaves,
                                                                  const int* nodes,
                                                                  const double* __restrict__ gin,
                                                                  int* counters) {
    __shared__ int next;
    const int per = (nwaves + 7) / 8;
    const int lo = (int)(blockIdx.x % 8) * per;
    const int hi = min(nwaves, lo + per);
    for (;;) {
        const int w0 = queue_take(counters, &next, lo);
        if (w0 >= hi) return;
        const int w1 = min(hi, w0 + kQueueChunk);
        for (int w = w0; w < w1; ++w) {
            if (w > w0) __syncthreads();
            const int2 d = waves[w];
            const AnalysisParams p = P[d.x];
            apply_node<N, T, MF>(p, nodes, d.y, gin);
        }
    }
}

// Blocks of a persistent launch: enough wavefronts to fill every CU (16 per CU,
// the most any of these kernels keeps resident), at most `items`; blocks
// beyond what fits start later and find the queue drained or nearly so.
inline int persistent_blocks(int threads, int items) {
    static int cus = 0;
    if (cus == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            cus = 256;
    }
    const int g = cus * 16 * 64 / threads;  // a multiple of 8: every XCD range has blocks
    return g < items ? g : items;           // items < g: one block per entry
}

template <int N>
hipError_t launch_n(const AnalysisParams& p, const int* nodes, int count, double* gbuf,
                    hipStream_t s) {
    if (count == 0) return hipSuccess;
    const size_t eig_bytes = (size_t)eig_lds_doubles<N>() * sizeof(double);
    const int segs = kSplitRows<N> ? 1 : EigLayout<N>::SEGS;
    const int eig_blocks = (count + segs - 1) / segs;
    static bool lds_ok = false;
    hipError_t e = allow_lds(analysis_eig_kernel<N>, eig_bytes, &lds_ok);
    if (e != hipSuccess) return e;
    analysis_eig_kernel<N><<<eig_blocks, eig_threads<N>(), eig_bytes, s>>>(p, nodes, count, gbuf);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t app_bytes = (size_t)apply_lds_doubles(N) * sizeof(double);
    if (p.storage == kStoreF32Dev && p.mfma_transform && kMfmaApply<N>)
        analysis_apply_kernel<N, float, true><<<count, 64, app_bytes, s>>>(p, nodes, count, gbuf);
    else if (p.storage == kStoreF32Dev)
        analysis_apply_kernel<N, float, false><<<count, 64, app_bytes, s>>>(p, nodes, count, gbuf);
    else
        analysis_apply_kernel<N, double, false><<<count, 64, app_bytes, s>>>(p, nodes, count, gbuf);
    return hipGetLastError();
}

template <int N>
hipError_t launch_batch_n(const AnalysisParams* d_params, const int4* d_eig_waves, int n_eig,
                          const int2* d_apply_waves, int n_apply, const int* d_nodes,
                          double* gbuf, int storage, bool mfma_transform, hipStream_t s) {
    if (n_eig == 0) return hipSuccess;
    const size_t eig_bytes = (size_t)eig_lds_doubles<N>() * sizeof(double);
    static bool lds_ok = false;
    hipError_t e = allow_lds(analysis_eig_batch_kernel<N>, eig_bytes, &lds_ok);
    if (e != hipSuccess) return e;
    analysis_eig_batch_kernel<N><<<n_eig, eig_threads<N>(), eig_bytes, s>>>(
        d_params, d_eig_waves, n_eig, d_nodes, gbuf);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t app_bytes = (size_t)apply_lds_doubles(N) * sizeof(double);
    if (storage == kStoreF32Dev && mfma_transform && kMfmaApply<N>)
        analysis_apply_batch_kernel<N, float, true><<<n_apply, 64, app_bytes, s>>>(
            d_params, d_apply_waves, n_apply, d_nodes, gbuf);
    else if (storage == kStoreF32Dev)
        analysis_apply_batch_kernel<N, float, false><<<n_apply, 64, app_bytes, s>>>(
            d_params, d_apply_waves, n_apply, d_nodes, gbuf);
    else
        analysis_apply_batch_kernel<N, double, false><<<n_apply, 64, app_bytes, s>>>(
            d_params, d_apply_waves, n_apply, d_nodes, gbuf);
    return hipGetLastError();
}

template <int N>
hipError_t launch_batch_queue_n(const AnalysisParams* d_params, const int4* d_eig_waves, int n_eig,
                                const int2* d_apply_waves, int n_apply, const int* d_nodes,
                                double* gbuf, int storage, bool mfma_transform, int* counters,
                                hipStream_t s) {
    if (n_eig == 0) return hipSuccess;
    const size_t eig_bytes = (size_t)eig_lds_doubles<N>() * sizeof(double);
    static bool lds_ok = false;
    hipError_t e = allow_lds(analysis_eig_queue_kernel<N>, eig_bytes, &lds_ok);
    if (e != hipSuccess) return e;
    const int ge = persistent_blocks(eig_threads<N>(), n_eig);
    analysis_eig_queue_kernel<N><<<ge, eig_threads<N>(), eig_bytes, s>>>(
        d_params, d_eig_waves, n_eig, d_nodes, gbuf, counters);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t app_bytes = (size_t)apply_lds_doubles(N) * sizeof(double);
    auto go = [&](auto kernel) {
        const int ga = persistent_blocks(64, n_apply);
        kernel<<<ga, 64, app_bytes, s>>>(d_params, d_apply_waves, n_apply, d_nodes, gbuf,
                                         counters + 8);
        return hipGetLastError();
    };
    if (storage == kStoreF32Dev && mfma_transform && kMfmaApply<N>)
        return go(analysis_apply_queue_kernel<N, float, true>);
    if (storage == kStoreF32Dev) return go(analysis_apply_queue_kernel<N, float, false>);
    return go(analysis_apply_queue_kernel<N, double, false>);
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
#define X(v) case v: return (eig_lds_doubles<v>() > apply_lds_doubles(v) ? eig_lds_doubles<v>() \
                                                                        : apply_lds_doubles(v)) * \
                            (int)sizeof(double);
        LBMLETKF_OBS_SIZES(X)
#undef X
        default: return 1 << 30;
    }
}

size_t obs_gbuf_doubles(int n, int count) { return (size_t)count * ((size_t)n * n + n); }

hipError_t launch_analysis_obs(const AnalysisParams& p, const int* nodes, int count, int n,
                               double* gbuf, hipStream_t s) {
    switch (n) {
#define X(v) case v: return launch_n<v>(p, nodes, count, gbuf, s);
        LBMLETKF_OBS_SIZES(X)
#undef X
        default: return hipErrorInvalidValue;
    }
}

namespace {
__global__ void zero_ints_kernel(int* v, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) v[i] = 0;
}
}  // namespace

hipError_t launch_zero_ints(int* v, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    zero_ints_kernel<<<1, 256, 0, s>>>(v, n);
    return hipGetLastError();
}

int obs_segments(int n) { return n > 0 ? 64 / n : 0; }

hipError_t launch_analysis_obs_batch_queue(const AnalysisParams* d_params, const int4* d_eig_waves,
                                           int n_eig, const int2* d_apply_waves, int n_apply,
                                           const int* d_nodes, int n, double* gbuf, int storage,
                                           bool mfma_transform, int* counters, hipStream_t s) {
    switch (n) {
#define X(v)                                                                                \
    case v:                                                                                 \
        return launch_batch_queue_n<v>(d_params, d_eig_waves, n_eig, d_apply_waves, n_apply, \
                                       d_nodes, gbuf, storage, mfma_transform, counters, s);
        LBMLETKF_OBS_SIZES(X)
#undef X
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_analysis_obs_batch(const AnalysisParams* d_params, const int4* d_eig_waves,
                                     int n_eig, const int2* d_apply_waves, int n_apply,
                                     const int* d_nodes, int n, double* gbuf, int storage,
                                     bool mfma_transform, hipStream_t s) {
    switch (n) {
#define X(v)                                                                                   \
    case v:                                                                                    \
        return launch_batch_n<v>(d_params, d_eig_waves, n_eig, d_apply_waves, n_apply, d_nodes, \
                                 gbuf, storage, mfma_transform, s);
        LBMLETKF_OBS_SIZES(X)
#undef X
        default: return hipErrorInvalidValue;
    }
}

}  // namespace lbmletkf
