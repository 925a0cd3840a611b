// Differentiation form: reverse-mode adjoint of the forecast (Sec. 2 LBE with
// BGK relaxation, Smagorinsky eddy viscosity, force and friction) and of the
// observation misfit J = sum_c sum_m sum_q (H_q(f_m(t_c)) - y^o_{c,q})^2.
//
// One forward step maps the canonical state f^n to f^{n+1} by
//     f^{n+1}_a(x) = C_a(f^n(x - c_a)),
// C the per-node collision.  Its adjoint is
//     lam^n_b(y) = sum_a lam^{n+1}_a(y + c_a) dC_a/df_b (f^n(y)),
// i.e. a push-direction gather of the adjoint and the transposed Jacobian of
// the collision at the forward state, written aligned.  The vector-Jacobian
// product below is the hand-derived reverse of the forward kernel's
// operations in reverse order (moments -> equilibrium -> non-equilibrium flux
// -> |Pi| -> tau -> omega, force with friction); it also returns the
// sensitivity to K = 18 sqrt(2) C_s^2, from which dJ/dC_s = (36 sqrt(2) C_s)
// * sum over steps, nodes and members.  At |Pi| = 0 the subgradient 0 is used.
#include "common.h"
#include "device_util.h"

namespace lbmletkf {
namespace {
using namespace dev;

constexpr int kBlock = 256;

// Reverse of one collision.  f: pre-collision populations; L: adjoint of the
// post-collision outputs.  Returns the adjoint of f in Lf and d(out.L)/dK.
__device__ __forceinline__ double collide_vjp(const double (&f)[9], const double (&L)[9],
                                              double tau0, double K, double fx_ext,
                                              double fy_ext, double mu, double (&Lf)[9]) {
    // ---- forward recomputation (same operations as the forward kernel)
    const double rho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
    const double jx = (f[1] - f[2]) + (f[5] - f[6]) + (f[7] - f[8]);
    const double jy = (f[3] - f[4]) + (f[5] - f[6]) + (f[8] - f[7]);
    const double ir = 1.0 / rho;
    const double u = jx * ir, v = jy * ir;
    const double pxx = (f[1] + f[2] + f[5] + f[6] + f[7] + f[8]) - rho * (1.0 / 3.0 + u * u);
    const double pyy = (f[3] + f[4] + f[5] + f[6] + f[7] + f[8]) - rho * (1.0 / 3.0 + v * v);
    const double pxy = (f[5] + f[6] - f[7] - f[8]) - rho * u * v;
    const double P = sqrt(pxx * pxx + pyy * pyy + 2.0 * pxy * pxy);
    const double R = sqrt(tau0 * tau0 + K * P * ir);
    const double tau = 0.5 * (tau0 + R);
    const double om = 1.0 / tau;
    const double gx = fx_ext - mu * u, gy = fy_ext - mu * v;
    const double usq = 1.5 * (u * u + v * v);
    double feq[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const double cu = cx_of(a) * u + cy_of(a) * v;
        feq[a] = rho * w_of(a) * (1.0 + 3.0 * cu + 4.5 * cu * cu - usq);
    }
    // ---- reverse
    double Lrho = 0.0, Lu = 0.0, Lv = 0.0, Lom = 0.0, Lgx = 0.0, Lgy = 0.0;
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const double cxa = cx_of(a), cya = cy_of(a), wa = w_of(a);
        Lf[a] = (1.0 - om) * L[a];                       // out_a = (1 - om) f_a + ...
        Lom += L[a] * (feq[a] - f[a]);                   // ... + om feq_a
        const double Lfeq = om * L[a];
        // F_a = 3 w rho (c.g)
        Lrho += L[a] * 3.0 * wa * (cxa * gx + cya * gy);
        Lgx += L[a] * 3.0 * wa * rho * cxa;
        Lgy += L[a] * 3.0 * wa * rho * cya;
        // feq_a = rho w (1 + 3 cu + 4.5 cu^2 - 1.5 u.u)
        const double cu = cxa * u + cya * v;
        Lrho += Lfeq * feq[a] * ir;
        Lu += Lfeq * rho * wa * (3.0 * cxa + 9.0 * cu * cxa - 3.0 * u);
        Lv += Lfeq * rho * wa * (3.0 * cya + 9.0 * cu * cya - 3.0 * v);
    }
    // g = F_ext - mu u
    Lu -= mu * Lgx;
    Lv -= mu * Lgy;
    // om = 1 / tau, tau = (tau0 + R) / 2, R = sqrt(tau0^2 + K P ir)
    const double Ltau = -Lom * om * om;
    const double Larg = 0.5 * Ltau / (2.0 * R);
    const double LP = Larg * K * ir;
    double Lir = Larg * K * P;
    const double LK = Larg * P * ir;
    // P = sqrt(pxx^2 + pyy^2 + 2 pxy^2)
    double Lpxx = 0.0, Lpyy = 0.0, Lpxy = 0.0;
    if (P > 0.0) {
        Lpxx = LP * pxx / P;
        Lpyy = LP * pyy / P;
        Lpxy = LP * 2.0 * pxy / P;
    }
    // pxx = sum cx^2 f - rho (1/3 + u^2), pyy likewise, pxy = sum cx cy f - rho u v
    Lrho -= Lpxx * (1.0 / 3.0 + u * u) + Lpyy * (1.0 / 3.0 + v * v) + Lpxy * u * v;
    Lu -= Lpxx * 2.0 * rho * u + Lpxy * rho * v;
    Lv -= Lpyy * 2.0 * rho * v + Lpxy * rho * u;
    // u = jx ir, v = jy ir, ir = 1 / rho
    const double Ljx = Lu * ir, Ljy = Lv * ir;
    Lir += Lu * jx + Lv * jy;
    Lrho -= Lir * ir * ir;
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const double cxa = cx_of(a), cya = cy_of(a);
        Lf[a] += Lrho + Ljx * cxa + Ljy * cya + Lpxx * cxa * cxa + Lpyy * cya * cya +
                 Lpxy * cxa * cya;
    }
    return LK;
}

// One reverse step, one thread per (node, member) as in the forward kernel.
// fstate: storage layout; lam_in, lam_out: adjoint states in the canonical
// node-major layout [node][a][member] (lam(y)_a of member m at slot(y, a, m)).
template <typename T>
__global__ __launch_bounds__(kBlock) void adjoint_step_kernel(
    const T* __restrict__ fstate, const double* __restrict__ lam_in, double* __restrict__ lam_out,
    const double* __restrict__ force, int nx, int ny, int members, double tau0, double K,
    double mu, double* __restrict__ k_partial) {
    const int plane = nx * ny;
    const int m = threadIdx.x;  // blockDim.x == members
    const int node = blockIdx.x * blockDim.y + threadIdx.y;
    double lk = 0.0;
    if (node < plane) {
        const int y = node / nx, x = node - y * nx;
        const int xm = wrap(x - 1, nx), xp = wrap(x + 1, nx);
        const int ym = wrap(y - 1, ny), yp = wrap(y + 1, ny);
        // forward state: canonical f_a(y) is held by the slot of node y - c_a
        const PullSlots<const T> fsrc(fstate, x, xm, xp, y, ym, yp, nx, members, m);
        // adjoint of f^{n+1}_a at the node this population streams to, y + c_a
        // (the same addressing with the neighbours swapped)
        const PullSlots<const double> lsrc(lam_in, x, xp, xm, y, yp, ym, nx, members, m);
        double f[9], L[9], Lf[9];
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            f[a] = PopIO<T>::load(fsrc.at(a), a);
            L[a] = *lsrc.at(a);
        }
        const double fx = force ? force[node] : 0.0, fy = force ? force[plane + node] : 0.0;
        lk = collide_vjp(f, L, tau0, K, fx, fy, mu, Lf);
        double* const out = lam_out + (size_t)node * 9 * members + m;
#pragma unroll
        for (int a = 0; a < 9; ++a) out[(uint32_t)a * members] = Lf[a];
    }
    // per-block sum of dJ/dK, accumulated in this block's own slot (launches
    // on one stream are ordered, so the accumulation is deterministic)
    const int tid = threadIdx.y * blockDim.x + threadIdx.x;
    const int nthreads = blockDim.x * blockDim.y;
    __shared__ double red[kBlock];
    if (nthreads % kWave == 0) {
        // whole wavefronts (M a power of two): a DPP sum per wavefront, then
        // the wavefront sums in order, one barrier
        const double ws = wave_sum(lk);
        if (tid % kWave == 0) red[tid / kWave] = ws;
        __syncthreads();
        if (tid == 0) {
            double t = 0.0;
            for (int w = 0; w < nthreads / kWave; ++w) t += red[w];
            k_partial[blockIdx.x] += t;
        }
        return;
    }
    red[tid] = lk;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (tid < s && tid + s < nthreads) red[tid] += red[tid + s];
        __syncthreads();
    }
    if (tid == 0) k_partial[blockIdx.x] += red[0];
}

// Misfit at one observation time.  One thread per (point, member), members
// fastest: adds (H - y^o)^2 to jbuf[m * npts + k] (if jbuf) and, if lam is
// given, dJ/df at the observation node to the adjoint state.
template <typename T>
__global__ void misfit_kernel(const T* __restrict__ f, const int* __restrict__ pts, int npts,
                              int nvar, const double* __restrict__ yo, double* __restrict__ lam,
                              double* __restrict__ jbuf, int nx, int ny, int members) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= npts * members) return;
    const int k = t / members, m = t - k * members;
    const int x = pts[2 * k], y = pts[2 * k + 1];
    double fa[9];
    double rho = 0.0, jx = 0.0, jy = 0.0;
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        fa[a] = PopIO<T>::load(f + slot(src_node(x, y, a, nx, ny), a, m, members), a);
        rho += fa[a];
        jx += cx_of(a) * fa[a];
        jy += cy_of(a) * fa[a];
    }
    const double u = jx / rho, v = jy / rho;
    const double* y0 = yo + (size_t)k * nvar;
    double rr = 0.0, ru = 0.0, rv = 0.0;
    if (nvar == 3) {
        rr = rho - y0[0];
        ru = u - y0[1];
        rv = v - y0[2];
    } else {
        ru = u - y0[0];
        rv = v - y0[1];
    }
    if (jbuf) jbuf[(size_t)m * npts + k] += rr * rr + ru * ru + rv * rv;
    if (lam) {
        // dJ/df_a = 2 rr + 2 ru (c_ax - u)/rho + 2 rv (c_ay - v)/rho
        const size_t node = (size_t)y * nx + x;
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            const double g = 2.0 * rr + 2.0 * (ru * (cx_of(a) - u) + rv * (cy_of(a) - v)) / rho;
            lam[slot(node, a, m, members)] += g;
        }
    }
}

// Adjoint state [node][a][member] -> canonical public layout [member][a][y][x].
__global__ void lam_to_canonical_kernel(const double* __restrict__ lam, double* __restrict__ out,
                                        int plane, int members) {
    const size_t total = (size_t)plane * 9 * members;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total;
         t += (size_t)gridDim.x * blockDim.x) {
        const size_t i = t % plane;
        const int a = (int)((t / plane) % 9);
        const int m = (int)(t / ((size_t)plane * 9));
        out[t] = lam[slot(i, a, m, members)];
    }
}

// Deterministic single-block sum of n doubles into out[0] (times scale).
__global__ __launch_bounds__(256) void sum_kernel(const double* __restrict__ v, size_t n,
                                                  double scale, double* __restrict__ out) {
    __shared__ double red[256];
    double s = 0.0;
    for (size_t i = threadIdx.x; i < n; i += 256) s += v[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = scale * red[0];
}

__global__ void fill_kernel(double* __restrict__ v, size_t n, double value) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        v[i] = value;
}

}  // namespace

int adjoint_partials(LbmDims d) {
    const int npb = nodes_per_block(d.members);
    return (d.nx * d.ny + npb - 1) / npb;
}

hipError_t launch_adjoint_step(const void* fstate, const double* lam_in, double* lam_out,
                               const double* force, LbmDims d, double tau0, double cs, double mu,
                               int storage, double* k_partial, hipStream_t s) {
    const int npb = nodes_per_block(d.members);
    const dim3 block(d.members, npb);
    const dim3 grid(adjoint_partials(d));
    const double K = 18.0 * sqrt(2.0) * cs * cs;
    if (storage == kStoreF32Dev)
        adjoint_step_kernel<float><<<grid, block, 0, s>>>((const float*)fstate, lam_in, lam_out,
                                                          force, d.nx, d.ny, d.members, tau0, K,
                                                          mu, k_partial);
    else
        adjoint_step_kernel<double><<<grid, block, 0, s>>>((const double*)fstate, lam_in,
                                                           lam_out, force, d.nx, d.ny, d.members,
                                                           tau0, K, mu, k_partial);
    return hipGetLastError();
}

hipError_t launch_lam_to_canonical(const double* lam, double* out, LbmDims d, hipStream_t s) {
    const size_t total = (size_t)d.nx * d.ny * 9 * d.members;
    size_t g = (total + 255) / 256;
    lam_to_canonical_kernel<<<(int)(g > 65536 ? 65536 : g), 256, 0, s>>>(lam, out, d.nx * d.ny,
                                                                         d.members);
    return hipGetLastError();
}

hipError_t launch_misfit(const void* f, const int* pts, int npts, int nvar, const double* yo,
                         double* lam, double* jbuf, LbmDims d, int storage, hipStream_t s) {
    const int total = npts * d.members;
    if (storage == kStoreF32Dev)
        misfit_kernel<float><<<(total + 127) / 128, 128, 0, s>>>((const float*)f, pts, npts, nvar,
                                                                 yo, lam, jbuf, d.nx, d.ny,
                                                                 d.members);
    else
        misfit_kernel<double><<<(total + 127) / 128, 128, 0, s>>>((const double*)f, pts, npts,
                                                                  nvar, yo, lam, jbuf, d.nx, d.ny,
                                                                  d.members);
    return hipGetLastError();
}

hipError_t launch_sum(const double* v, size_t n, double scale, double* out, hipStream_t s) {
    sum_kernel<<<1, 256, 0, s>>>(v, n, scale, out);
    return hipGetLastError();
}

hipError_t launch_fill(double* v, size_t n, double value, hipStream_t s) {
    size_t g = (n + 255) / 256;
    fill_kernel<<<(int)(g > 65536 ? 65536 : (g == 0 ? 1 : g)), 256, 0, s>>>(v, n, value);
    return hipGetLastError();
}

}  // namespace lbmletkf
