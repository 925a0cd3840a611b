// Device helpers shared by the analysis translation units: wave reductions,
// intra-wave LDS ordering, periodic wrap, XCD-aware block order and the
// segmented parallel Jacobi eigensolver.
#pragma once
#include "common.h"

namespace lbmletkf {
namespace dev {

// ---------------------------------------------------------------------------
// reductions over aligned groups of G lanes (G a power of two <= 64), on the
// VALU: a butterfly inside each row of 16 lanes with DPP moves (xor 1 and
// xor 2 as quad permutations; then the half-row and row mirrors, which pair
// the same quads and half-rows as xor 4 and xor 8 once every quad, then every
// half-row, holds one value), and for G = 32, 64 the row results read with
// v_readlane and combined in a fixed order.  Every lane of a group gets the
// same bits.  Call in wave-uniform control flow (all 64 lanes active).
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ double dpp_partner(double x) {
    // every source lane of these patterns lies in the row, so bound_ctrl (zero
    // for an out-of-row source) never applies; it spares initialising the result
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double lane_value(double x, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
    return __hiloint2double(hi, lo);
}

template <int G, typename Op>
__device__ __forceinline__ double group_reduce(double x, Op op) {
    static_assert(G >= 1 && G <= 64 && (G & (G - 1)) == 0, "group size must be a power of two");
    if (G >= 2) x = op(x, dpp_partner<0xB1>(x));   // quad_perm [1, 0, 3, 2]
    if (G >= 4) x = op(x, dpp_partner<0x4E>(x));   // quad_perm [2, 3, 0, 1]
    if (G >= 8) x = op(x, dpp_partner<0x141>(x));  // row_half_mirror
    if (G >= 16) x = op(x, dpp_partner<0x140>(x)); // row_mirror
    if (G == 32) {
        const double lo = op(lane_value(x, 0), lane_value(x, 16));
        const double hi = op(lane_value(x, 32), lane_value(x, 48));
        x = (threadIdx.x & 32) ? hi : lo;
    } else if (G == 64) {
        x = op(op(op(lane_value(x, 0), lane_value(x, 16)), lane_value(x, 32)), lane_value(x, 48));
    }
    return x;
}

struct OpAdd {
    __device__ double operator()(double a, double b) const { return a + b; }
};
struct OpMin {
    __device__ double operator()(double a, double b) const { return fmin(a, b); }
};
struct OpMax {
    __device__ double operator()(double a, double b) const { return fmax(a, b); }
};

__device__ __forceinline__ double wave_sum(double v) { return group_reduce<kWave>(v, OpAdd()); }

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
// wave-level parallel Jacobi on SEGS independent N x N symmetric matrices
// (N even).  Lane l belongs to segment seg = l / N and holds row i = l % N of
// its matrix S and of the accumulated rotation matrix U in registers.
// Round P rotates the pairs (2k+P, 2k+P+1) and swaps them (Brent-Luk
// ordering): rows are published to LDS, both lanes of a pair read a_pp,
// a_qq, a_pq from there (so they derive bit-identical rotations), the row
// mix reads the partner's pre-round row from LDS, and the column mix of S
// and U is in-register with the pair's (c, s) read back from LDS.
// ---------------------------------------------------------------------------
template <int N>
__device__ __forceinline__ double extract_lane_entry(const double (&R)[N], int col) {
    double v = 0.0;
#pragma unroll
    for (int r = 0; r < N; ++r) v = (r == col) ? R[r] : v;
    return v;
}

// Row stride (doubles) of the Jacobi row exchange: 16 lanes reading 16-byte
// pieces of consecutive rows hit distinct LDS banks when stride/2 is odd.
template <int N>
struct RowStride {
    static constexpr int value = (N % 4 == 2) ? N : N + 2;
};

// Rotation (c, s) that annihilates a_pq of the 2 x 2 block [[a_pp, a_pq], [a_pq, a_qq]]
// (c = 1, s = 0 for a_pq = 0 or when `use` is false).
// t = sgn(tau) / (|tau| + sqrt(1 + tau^2)),
// tau = (a_qq - a_pp) / (2 a_pq), the smaller root of t^2 + 2 tau t - 1 = 0:
// tau from the hardware FP64 reciprocal of a_pq (no overflow or underflow
// short of FP64's range), then t in FP32.  Any t gives an exactly orthogonal
// rotation through c and s below (FP64), and an FP32-accurate t still removes
// all but ~1e-7 of a_pq, which the next sweeps finish.  |tau| beyond FP32's
// range converts to inf and gives t = 0 (a_pq negligible against a_qq - a_pp).
// Branch-free: for a_pq = 0 the intermediate t is inf or NaN and the final
// select discards it, so the three operand loads of a caller issue together
// instead of waiting on a test of a_pq.
__device__ __forceinline__ void jacobi_rotation(double app, double aqq, double apq, bool use,
                                                double* cp, double* sp) {
    const double d = aqq - app;
    const float tau = (float)(d * (0.5 * __builtin_amdgcn_rcp(apq)));
    const float at = fabsf(tau);
    // |tau| + sqrt(1 + tau^2), or 2 |tau| where tau^2 would overflow
    const float den = at > 1e18f ? at + at : at + __builtin_amdgcn_sqrtf(1.0f + at * at);
    const float tf = copysignf(__builtin_amdgcn_rcpf(den), tau);
    const double t = (double)tf;
    const double c = rsqrt(1.0 + t * t);
    const bool rot = use && apq != 0.0;
    *cp = rot ? c : 1.0;
    *sp = rot ? t * c : 0.0;
}

template <int N, int SEGS, int P>
__device__ __forceinline__ void jacobi_round(double (&S)[N], double (&U)[N], double* rows,
                                             double2* cs, int lane) {
    constexpr int RS = RowStride<N>::value;
    const int seg = lane / N;
    const int i = lane - seg * N;
    const bool active = seg < SEGS;
    const int sbase = active ? seg * N : 0;
    double* segrows = rows + (size_t)sbase * RS;
    // publish this lane's row
    wave_lds_sync();
    if (active) {
        double2* my = reinterpret_cast<double2*>(segrows + (size_t)i * RS);
#pragma unroll
        for (int k = 0; k < N / 2; ++k) my[k] = make_double2(S[2 * k], S[2 * k + 1]);
    }
    wave_lds_sync();
    const bool first = ((i - P) & 1) == 0;
    const int pi = first ? i + 1 : i - 1;
    const bool paired = active && pi >= 0 && pi < N;
    // a lane without a partner reads the first pair's block and discards it
    const int p = paired ? (first ? i : pi) : 0;
    const double2* pr = reinterpret_cast<const double2*>(segrows + (size_t)(paired ? pi : i) * RS);
    // the first four slices of the partner's row are read with the block, so
    // that their latency hides behind the rotation's arithmetic (N = 24: 169 ->
    // 167 VGPRs, three wavefronts per SIMD instead of two)
    constexpr int KP = N / 2 < 4 ? N / 2 : 4;
    double2 pre[KP];
#pragma unroll
    for (int k = 0; k < KP; ++k) pre[k] = pr[k];
    double c, s;
    jacobi_rotation(segrows[(size_t)p * RS + p], segrows[(size_t)(p + 1) * RS + p + 1],
                    segrows[(size_t)p * RS + p + 1], paired, &c, &s);
    cs[lane] = make_double2(c, s);
    wave_lds_sync();
    // S <- P^T J^T S J P and U <- U J P, one double2 of the row at a time, so
    // that only a slice of the partner's row and of the (c, s) list is live:
    // the row mix of entries 2k, 2k+1 (from the partner's row as published; a
    // lane without a partner takes its own row with c = 1, s = 0, which leaves
    // it unchanged), then the column rotation of each pair (r, r+1) whose two
    // entries are mixed, by the pair's (c, s)
    const double sg = first ? s : -s;
#pragma unroll
    for (int k = 0; k < N / 2; ++k) {
        const double2 v = k < KP ? pre[k < KP ? k : 0] : pr[k];
        S[2 * k] = c * v.x + sg * S[2 * k];
        S[2 * k + 1] = c * v.y + sg * S[2 * k + 1];
        const int r = 2 * k - P;
        if (r >= 0) {
            const double2 q = cs[sbase + r];
            const double a0 = S[r], a1 = S[r + 1];
            S[r] = q.y * a0 + q.x * a1;
            S[r + 1] = q.x * a0 - q.y * a1;
            const double u0 = U[r], u1 = U[r + 1];
            U[r] = q.y * u0 + q.x * u1;
            U[r + 1] = q.x * u0 - q.y * u1;
        }
    }
    // pin this round's U rotations here: otherwise the compiler sinks them into
    // the next round, next to their first use, which keeps every (c, s) of
    // the round live (about N more doubles per lane) and costs occupancy
#pragma unroll
    for (int r = 0; r < N; ++r) asm volatile("" : "+v"(U[r]), "+v"(S[r]));
}

// Sweeps until every segment's off-diagonal Frobenius norm is below 1e-13
// of its diagonal norm.  Returns the sweeps used, max_sweeps + 1 if a segment
// did not converge.  `red` holds 2 doubles per lane.
template <int N, int SEGS>
__device__ int jacobi_eig(double (&S)[N], double (&U)[N], double* rows, double2* cs,
                          double* red, int lane, int max_sweeps) {
    const int seg = lane / N;
    const int i = lane - seg * N;
    const bool active = seg < SEGS;
    const int sbase = active ? seg * N : 0;
    for (int sweep = 0;; ++sweep) {
        double off = 0.0, dg = 0.0;
#pragma unroll
        for (int r = 0; r < N; ++r) {
            const double v2 = S[r] * S[r];
            if (r == i) dg += v2; else off += v2;
        }
        wave_lds_sync();
        red[2 * lane] = active ? off : 0.0;
        red[2 * lane + 1] = active ? dg : 0.0;
        wave_lds_sync();
        double so = 0.0, sd = 0.0;
        for (int k = 0; k < N; ++k) {
            so += red[2 * (sbase + k)];
            sd += red[2 * (sbase + k) + 1];
        }
        const bool done = !active || so <= 1e-26 * sd;
        if (__all(done)) return sweep;
        if (sweep >= max_sweeps) return max_sweeps + 1;
#pragma unroll 1
        for (int rr = 0; rr < N / 2; ++rr) {
            jacobi_round<N, SEGS, 0>(S, U, rows, cs, lane);
            jacobi_round<N, SEGS, 1>(S, U, rows, cs, lane);
        }
    }
}

// ---------------------------------------------------------------------------
// The same parallel Jacobi with skewed rows: lane i (row i, segment base
// b = i rounded down to even) keeps column (b + k) mod N of its rows of S and
// U in register k.  Both lanes of a pair (2m, 2m + 1) then hold the same
// columns in the same registers, and a_pp, a_pq, a_qq of their 2 x 2 block sit
// in registers 0 and 1, so a P = 0 round takes the partner's row and the block
// by DPP quad permutations instead of through LDS; only the rotations (c, s)
// go through LDS, to every lane of the segment.  P = 1 rounds publish each
// row through LDS where its partner reads it.  Every entry sees the same
// operations on the same operands as in the unskewed solver, up to exact sign
// changes.
// ---------------------------------------------------------------------------
// Row stride (doubles) of a skewed published row: an odd lane's registers at
// 0..N-1 (0, 1 again at N, N+1), an even lane's at 4..N+3 (N-2, N-1 again at
// 2, 3), so that every partner reads at offset 2; stride/2 odd.
template <int N>
struct SkewStride {
    static constexpr int value = (N % 4 == 2) ? N + 4 : N + 6;
};

// (c, s) lists of the skewed solver, one entry per pair: pair m of a round is
// columns (2m + P, 2m + P + 1) (for P = 1, m = N/2 - 1 stands for the unpaired
// columns N - 1, 0), and entry m + N/2 repeats entry m, so that register pair j
// of a lane with base b reads entry b/2 + j without a wrap.  Segments start
// skew_cs_stride(N) entries apart: with 16 lanes per LDS pass and 64 banks the
// entries the active lanes of one read instruction touch then fall on distinct
// banks.
__host__ __device__ constexpr int skew_cs_stride(int n) {
    return n == 10 ? 21 : n == 14 ? 23 : n == 18 ? 25 : n == 20 ? 26 : n == 22 ? 29
         : n == 24 ? 28 : n == 26 ? 29 : n == 28 ? 30 : n == 30 ? 31 : n == 12 ? 13 : n;
}
template <int N, int SEGS>
__host__ __device__ constexpr int skew_cs_doubles() { return SEGS * skew_cs_stride(N) * 2; }

template <int N, int SEGS, int P>
__device__ __forceinline__ void jacobi_round_skew(double (&S)[N], double (&U)[N], double* rows,
                                                  double2* cs2, int lane) {
    constexpr int RS = SkewStride<N>::value;
    const int seg = lane / N;
    const int i = lane - seg * N;
    const bool active = seg < SEGS;
    const int sbase = active ? seg * N : 0;
    const bool odd = (i & 1) != 0;
    const int base = i - (i & 1);
    double2* csl = cs2 + (size_t)(active ? seg : 0) * skew_cs_stride(N);
    const int hb = base / 2;
    const bool first = ((i - P) & 1) == 0;
    double c, s;
    if constexpr (P == 0) {
        // block [[a_pp, a_pq], [a_pq, a_qq]] of pair (2m, 2m + 1): a_pp, a_pq from
        // the even lane's registers 0, 1 and a_qq from the odd lane's register 1,
        // the same values in both lanes
        const double x0 = dpp_partner<0xB1>(S[0]);
        const double x1 = dpp_partner<0xB1>(S[1]);
        const double app = odd ? x0 : S[0];
        const double apq = odd ? x1 : S[1];
        const double aqq = odd ? S[1] : x1;
        jacobi_rotation(app, aqq, apq, active, &c, &s);
        wave_lds_sync();
        if (active && !odd) {
            csl[i / 2] = make_double2(c, s);
            csl[i / 2 + N / 2] = make_double2(c, s);
        }
        // row mix with the partner's row (same columns, same registers)
        const double sg = first ? s : -s;
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const double v = dpp_partner<0xB1>(S[k]);
            S[k] = c * v + sg * S[k];
        }
        wave_lds_sync();
        // column rotation of each pair: registers (2j, 2j + 1) hold columns
        // (b + 2j, b + 2j + 1) mod N, an even first column
#pragma unroll
        for (int j = 0; j < N / 2; ++j) {
            const double2 q = csl[hb + j];
            const int r = 2 * j;
            const double a0 = S[r], a1 = S[r + 1];
            S[r] = q.y * a0 + q.x * a1;
            S[r + 1] = q.x * a0 - q.y * a1;
            const double u0 = U[r], u1 = U[r + 1];
            U[r] = q.y * u0 + q.x * u1;
            U[r + 1] = q.x * u0 - q.y * u1;
        }
    } else {
        double* segrows = rows + (size_t)sbase * RS;
        wave_lds_sync();
        // Each lane publishes its row where its partner reads it at offset 2:
        // column b + k of an odd lane's partner (base b + 2) is that lane's
        // register k - 2, of an even lane's partner (base b - 2) its register
        // k + 2.  So an odd lane stores register r at r (and registers 0, 1
        // again at N, N + 1), an even lane at r + 4 (and registers N - 2, N - 1
        // again at 2, 3).
        if (active) {
            double2* my = reinterpret_cast<double2*>(segrows + (size_t)i * RS + (odd ? 0 : 4));
#pragma unroll
            for (int k = 0; k < N / 2; ++k) my[k] = make_double2(S[2 * k], S[2 * k + 1]);
            *reinterpret_cast<double2*>(segrows + (size_t)i * RS + (odd ? N : 2)) =
                odd ? make_double2(S[0], S[1]) : make_double2(S[N - 2], S[N - 1]);
        }
        wave_lds_sync();
        // pair (2m + 1, 2m + 2): a_pp, a_pq are the odd lane's registers 1, 2
        // (stored at 1, 2), a_qq the even lane's register 0 (stored at 4); a lane
        // without a partner reads the first pair's block and discards it
        const int pi = first ? i + 1 : i - 1;
        const bool paired = active && pi >= 0 && pi < N;
        const int p = paired ? (first ? i : pi) : 1;
        // a lane without a partner reads its own row and keeps (lane 0:
        // negates) its own values: coefficients (0, 1), (0, -1) below
        const int src = paired ? pi : (active ? i : 0);
        const double2* pr = reinterpret_cast<const double2*>(segrows + (size_t)src * RS + 2);
        constexpr int KP = N / 2 < 4 ? N / 2 : 4;
        double2 pre[KP];
#pragma unroll
        for (int k = 0; k < KP; ++k) pre[k] = pr[k];
        jacobi_rotation(segrows[(size_t)p * RS + 1], segrows[(size_t)(p + 1) * RS + 4],
                        segrows[(size_t)p * RS + 2], paired, &c, &s);
        // Columns N - 1 and 0, which no rotation pairs in this round, meet in
        // registers (N - 1 - b, N - b) of every lane, where the pair update
        // (which swaps as it rotates) runs on them too.  The list entry of
        // column N - 1, (c, s) = (0, 1), makes that update keep column N - 1
        // and negate column 0: S D, U D with D = diag(-1, 1, ..., 1).  Lane 0
        // negates its row (below), which completes D S D, a similarity; the negations
        // are exact, so every entry keeps the magnitude the unskewed solver
        // gives it, and the eigenvectors change sign only.
        if (active && odd) {
            const double2 q = i == N - 1 ? make_double2(0.0, 1.0) : make_double2(c, s);
            csl[i / 2] = q;
            csl[i / 2 + N / 2] = q;
        }
        wave_lds_sync();
        const double cr = paired ? c : 0.0;
        const double sg = paired ? (first ? s : -s) : ((active && i == 0) ? -1.0 : 1.0);
#pragma unroll
        for (int k = 0; k < N / 2; ++k) {
            const double2 v = k < KP ? pre[k < KP ? k : 0] : pr[k];
            S[2 * k] = cr * v.x + sg * S[2 * k];
            S[2 * k + 1] = cr * v.y + sg * S[2 * k + 1];
        }
        // column pairs (odd first column): registers (k, k + 1) for odd k, and
        // (N - 1, 0)
#pragma unroll
        for (int j = 0; j < N / 2; ++j) {
            const int r0 = 2 * j + 1, r1 = (2 * j + 2) % N;
            const double2 q = csl[hb + j];
            const double a0 = S[r0], a1 = S[r1];
            S[r0] = q.y * a0 + q.x * a1;
            S[r1] = q.x * a0 - q.y * a1;
            const double u0 = U[r0], u1 = U[r1];
            U[r0] = q.y * u0 + q.x * u1;
            U[r1] = q.x * u0 - q.y * u1;
        }
    }
#pragma unroll
    for (int r = 0; r < N; ++r) asm volatile("" : "+v"(U[r]), "+v"(S[r]));
}

// Skewed-row Jacobi: S comes in unskewed (lane i holds row i, register c
// column c), U is set to the identity, and both go out unskewed; `rows` needs
// max(SEGS * N * SkewStride<N>, 128) doubles (the rows, and the convergence
// partial sums between sweeps), `cs2` skew_cs_doubles<N, SEGS>() doubles.
template <int N, int SEGS>
__device__ int jacobi_eig_skew(double (&S)[N], double (&U)[N], double* rows, double2* cs2,
                               int lane, int max_sweeps) {
    constexpr int RS = SkewStride<N>::value;
    const int seg = lane / N;
    const int i = lane - seg * N;
    const bool active = seg < SEGS;
    const int sbase = active ? seg * N : 0;
    const bool odd = (i & 1) != 0;
    const int base = i - (i & 1);
    double* myrow = rows + (size_t)(sbase + (active ? i : 0)) * RS;
    // skew S through LDS; U = I skewed: column i sits in register i - b
    wave_lds_sync();
    if (active) {
#pragma unroll
        for (int k = 0; k < N; ++k) myrow[k] = S[k];
    }
    wave_lds_sync();
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const int cidx = base + k < N ? base + k : base + k - N;
        S[k] = active ? myrow[cidx] : 0.0;
        U[k] = 0.0;
    }
    U[0] = (active && !odd) ? 1.0 : 0.0;
    U[1] = (active && odd) ? 1.0 : 0.0;
    int result = -1;
    for (int sweep = 0;; ++sweep) {
        const double d0 = S[0] * S[0], d1 = S[1] * S[1];
        double off = odd ? d0 : d1;
        const double dg = odd ? d1 : d0;
#pragma unroll
        for (int r = 2; r < N; ++r) off += S[r] * S[r];
        wave_lds_sync();
        rows[2 * lane] = active ? off : 0.0;
        rows[2 * lane + 1] = active ? dg : 0.0;
        wave_lds_sync();
        double so = 0.0, sd = 0.0;
        for (int k = 0; k < N; ++k) {
            so += rows[2 * (sbase + k)];
            sd += rows[2 * (sbase + k) + 1];
        }
        const bool done = !active || so <= 1e-26 * sd;
        if (__all(done)) { result = sweep; break; }
        if (sweep >= max_sweeps) { result = max_sweeps + 1; break; }
#pragma unroll 1
        for (int rr = 0; rr < N / 2; ++rr) {
            jacobi_round_skew<N, SEGS, 0>(S, U, rows, cs2, lane);
            jacobi_round_skew<N, SEGS, 1>(S, U, rows, cs2, lane);
        }
    }
    // unskew S, then U, through LDS
    wave_lds_sync();
    if (active) {
#pragma unroll
        for (int k = 0; k < N; ++k) myrow[base + k < N ? base + k : base + k - N] = S[k];
    }
    wave_lds_sync();
#pragma unroll
    for (int k = 0; k < N; ++k) S[k] = active ? myrow[k] : 0.0;
    wave_lds_sync();
    if (active) {
#pragma unroll
        for (int k = 0; k < N; ++k) myrow[base + k < N ? base + k : base + k - N] = U[k];
    }
    wave_lds_sync();
#pragma unroll
    for (int k = 0; k < N; ++k) U[k] = active ? myrow[k] : 0.0;
    wave_lds_sync();
    return result;
}

// One node's cycle-diagnostics record from the group of G lanes (the whole
// wavefront by default) that holds the node (lane = member, lanes >= M hold
// nothing): the squared error of the
// ensemble-mean velocity against the truth (0 without truth), the spread
// sum_m |u_m - u_bar|^2 / (M - 1), the number of members with a non-finite
// density or velocity, and the density range; lane 0 writes the five fields
// to out[0..4].  The same quantities, per node, as diag_partial_kernel.
template <int G = kWave>
__device__ __forceinline__ void node_diag_record(const double (&f)[9], bool mem, int M, int node,
                                                 int plane, const double* truth_uv, double* out) {
    double u = 0.0, v = 0.0, rho = 1.0, bad = 0.0, rmin = INFINITY, rmax = -INFINITY;
    if (mem) {
        double jx = 0.0, jy = 0.0;
        rho = 0.0;
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            rho += f[a];
            jx += cx_of(a) * f[a];
            jy += cy_of(a) * f[a];
        }
        u = jx / rho;
        v = jy / rho;
        if (!isfinite(rho) || !isfinite(u) || !isfinite(v)) bad = 1.0;
        rmin = rho;
        rmax = rho;
    }
    auto gsum = [](double x) { return group_reduce<G>(x, OpAdd()); };
    const double ub = gsum(u) / M, vb = gsum(v) / M;
    double err2 = 0.0, spr2 = 0.0;
    if (truth_uv) {
        const double du = ub - truth_uv[node], dv = vb - truth_uv[plane + node];
        err2 = du * du + dv * dv;
    }
    if (M > 1) {
        const double du = mem ? u - ub : 0.0, dv = mem ? v - vb : 0.0;
        spr2 = gsum(du * du + dv * dv) / (M - 1);
    }
    bad = gsum(bad);
    rmin = group_reduce<G>(rmin, OpMin());
    rmax = group_reduce<G>(rmax, OpMax());
    if (threadIdx.x % G == 0) {
        out[0] = err2;
        out[1] = spr2;
        out[2] = bad;
        out[3] = rmin;
        out[4] = rmax;
    }
}

// Block b runs on XCD b % 8; give each XCD a contiguous range of work items
// so that nodes sharing cache lines meet in the same L2.
__device__ __forceinline__ int xcd_remap(int b, int nblocks) {
    const int per = nblocks / 8;
    if (b >= per * 8) return b;
    return (b % 8) * per + b / 8;
}

}  // namespace dev
}  // namespace lbmletkf
