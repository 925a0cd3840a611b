// Forecast kernels: the D2Q9 lattice Boltzmann equation with BGK relaxation,
// Smagorinsky eddy viscosity and a body force (Sec. 2), advanced for every
// ensemble member in one launch.
//
// Layout: SoA f[member][a][y][x], FP64, x fastest.  The kernels pull: the
// thread of node (x, y) gathers f_a from (x - c_a, y - c_a), which is the
// pre-collision population f_a(x, y, t), collides, and writes f*_a to its own
// slot (a, y, x).  Between steps a buffer therefore holds post-collision
// values, and the canonical f_a(x, y) lives at slot (a, y - c_ay, x - c_ax);
// import/export convert.  Every load and store is coalesced along x (the x
// shift only misaligns rows by one element).
//
// Relaxation time: the strain rate is taken from the local non-equilibrium
// momentum flux Pi = sum_a c_a c_a (f_a - f_a^eq) through the Chapman-Enskog
// relation S = -3 Pi / (2 rho tau); with nu + nu_SGS = (tau - 1/2)/3 and
// nu_SGS = C_s^2 |S| (Sec. 2) tau solves
//     tau^2 - tau0 tau - 9 sqrt(2) C_s^2 |Pi| / (2 rho) = 0,
// |Pi| = sqrt(Pi_xx^2 + Pi_yy^2 + 2 Pi_xy^2), whose positive root is used.
// The momentum flux of f^eq is rho/3 I + rho u u, so Pi needs no f^eq.
#include "common.h"

namespace lbmletkf {
namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ int wrap_dec(int i, int n) { return i == 0 ? n - 1 : i - 1; }
__device__ __forceinline__ int wrap_inc(int i, int n) { return i == n - 1 ? 0 : i + 1; }

// Relax one node: f[9] in (pre-collision), f*[9] out.
__device__ __forceinline__ void collide_node(double (&f)[9], double tau0, double smag,
                                             double fx_ext, double fy_ext, double mu) {
    const double rho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
    const double jx = (f[1] - f[2]) + (f[5] - f[6]) + (f[7] - f[8]);
    const double jy = (f[3] - f[4]) + (f[5] - f[6]) + (f[8] - f[7]);
    const double inv_rho = 1.0 / rho;
    const double u = jx * inv_rho, v = jy * inv_rho;
    const double uu = u * u, vv = v * v, uv = u * v;
    // non-equilibrium momentum flux
    const double pxx = (f[1] + f[2] + f[5] + f[6] + f[7] + f[8]) - rho * (1.0 / 3.0 + uu);
    const double pyy = (f[3] + f[4] + f[5] + f[6] + f[7] + f[8]) - rho * (1.0 / 3.0 + vv);
    const double pxy = (f[5] + f[6] - f[7] - f[8]) - rho * uv;
    const double pn = sqrt(pxx * pxx + pyy * pyy + 2.0 * pxy * pxy);
    const double tau = 0.5 * (tau0 + sqrt(tau0 * tau0 + smag * pn * inv_rho));
    const double omega = 1.0 / tau;
    // acceleration: external field plus linear friction
    const double gx = fx_ext - mu * u, gy = fy_ext - mu * v;
    const double usq = 1.5 * (uu + vv);
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const double cu = cx_of(a) * u + cy_of(a) * v;
        const double feq = rho * w_of(a) * (1.0 + 3.0 * cu + 4.5 * cu * cu - usq);
        const double Fa = 3.0 * w_of(a) * rho * (cx_of(a) * gx + cy_of(a) * gy);
        f[a] = f[a] - omega * (f[a] - feq) + Fa;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void stream_collide_kernel(
    const T* __restrict__ fin, T* __restrict__ fout, const double* __restrict__ force, int nx,
    int ny, double tau0, double smag, double mu) {
    const int plane = nx * ny;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= plane) return;
    const int m = blockIdx.y;
    const int y = i / nx, x = i - y * nx;
    const int xm = wrap_dec(x, nx), xp = wrap_inc(x, nx);
    const int ym = wrap_dec(y, ny), yp = wrap_inc(y, ny);
    const T* __restrict__ b = fin + (size_t)m * 9 * plane;
    const int rc = y * nx, rm = ym * nx, rp = yp * nx;
    // every population is read once and written once per step: stream it
    // past the caches (nontemporal loads and stores)
    const size_t src[9] = {(size_t)rc + x,
                           (size_t)1 * plane + rc + xm,
                           (size_t)2 * plane + rc + xp,
                           (size_t)3 * plane + rm + x,
                           (size_t)4 * plane + rp + x,
                           (size_t)5 * plane + rm + xm,
                           (size_t)6 * plane + rp + xp,
                           (size_t)7 * plane + rp + xm,
                           (size_t)8 * plane + rm + xp};
    double f[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) f[a] = PopIO<T>::load_nt(b + src[a], a);
    double fx = 0.0, fy = 0.0;
    if (force) {
        fx = force[i];
        fy = force[plane + i];
    }
    collide_node(f, tau0, smag, fx, fy, mu);
    T* __restrict__ o = fout + (size_t)m * 9 * plane + i;
#pragma unroll
    for (int a = 0; a < 9; ++a) PopIO<T>::store_nt(o + (size_t)a * plane, a, f[a]);
}

// storage slot (a, y, x) <- canonical (a, y + c_ay, x + c_ax)
template <typename T>
__global__ void import_kernel(const double* __restrict__ canon, T* __restrict__ f, int nx,
                              int ny, int members) {
    const size_t plane = (size_t)nx * ny;
    const size_t total = plane * 9 * members;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total;
         t += (size_t)gridDim.x * blockDim.x) {
        const size_t i = t % plane;
        const int a = (int)((t / plane) % 9);
        const int y = (int)(i / nx), x = (int)(i % nx);
        const int xs = (x + cx_of(a) + nx) % nx, ys = (y + cy_of(a) + ny) % ny;
        PopIO<T>::store(f + t, a, canon[t - i + (size_t)ys * nx + xs]);
    }
}

// canonical (a, y, x) <- storage slot (a, y - c_ay, x - c_ax)
template <typename T>
__global__ void export_kernel(const T* __restrict__ f, double* __restrict__ canon, int nx,
                              int ny, int members) {
    const size_t plane = (size_t)nx * ny;
    const size_t total = plane * 9 * members;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total;
         t += (size_t)gridDim.x * blockDim.x) {
        const size_t i = t % plane;
        const int a = (int)((t / plane) % 9);
        const int y = (int)(i / nx), x = (int)(i % nx);
        const int xs = (x - cx_of(a) + nx) % nx, ys = (y - cy_of(a) + ny) % ny;
        canon[t] = PopIO<T>::load(f + (t - i + (size_t)ys * nx + xs), a);
    }
}

// f^eq(rho, u) written to the storage slots of node (x, y).
template <typename T>
__global__ void init_equilibrium_kernel(const double* __restrict__ rho_in,
                                        const double* __restrict__ uv, T* __restrict__ f, int nx,
                                        int ny, int members) {
    const size_t plane = (size_t)nx * ny;
    const size_t total = plane * members;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total;
         t += (size_t)gridDim.x * blockDim.x) {
        const size_t i = t % plane;
        const size_t m = t / plane;
        const int y = (int)(i / nx), x = (int)(i % nx);
        const double rho = rho_in ? rho_in[t] : 1.0;
        const double u = uv[(m * 2) * plane + i], v = uv[(m * 2 + 1) * plane + i];
        const double usq = 1.5 * (u * u + v * v);
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            const double cu = cx_of(a) * u + cy_of(a) * v;
            const int xs = (x - cx_of(a) + nx) % nx, ys = (y - cy_of(a) + ny) % ny;
            PopIO<T>::store(f + ((m * 9 + a) * plane + (size_t)ys * nx + xs), a,
                            rho * w_of(a) * (1.0 + 3.0 * cu + 4.5 * cu * cu - usq));
        }
    }
}

// rho, u, v of every node from the canonical populations.
template <typename T>
__global__ void moments_kernel(const T* __restrict__ f, double* __restrict__ out, int nx,
                               int ny, int members) {
    const size_t plane = (size_t)nx * ny;
    const size_t total = plane * members;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total;
         t += (size_t)gridDim.x * blockDim.x) {
        const size_t i = t % plane;
        const size_t m = t / plane;
        const int y = (int)(i / nx), x = (int)(i % nx);
        double rho = 0.0, jx = 0.0, jy = 0.0;
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            const int xs = (x - cx_of(a) + nx) % nx, ys = (y - cy_of(a) + ny) % ny;
            const double fa = PopIO<T>::load(f + ((m * 9 + a) * plane + (size_t)ys * nx + xs), a);
            rho += fa;
            jx += cx_of(a) * fa;
            jy += cy_of(a) * fa;
        }
        out[(m * 3) * plane + i] = rho;
        out[(m * 3 + 1) * plane + i] = jx / rho;
        out[(m * 3 + 2) * plane + i] = jy / rho;
    }
}

int grid_for(size_t total, int block) {
    size_t g = (total + block - 1) / block;
    return (int)(g > 65536 ? 65536 : (g == 0 ? 1 : g));
}

}  // namespace

hipError_t launch_stream_collide(const void* fin, void* fout, const double* force, LbmDims d,
                                 double tau0, double cs, double mu, int storage, hipStream_t s) {
    const int plane = d.nx * d.ny;
    dim3 grid((plane + kBlock - 1) / kBlock, d.members);
    const double smag = 18.0 * sqrt(2.0) * cs * cs;
    if (storage == kStoreF32Dev)
        stream_collide_kernel<float><<<grid, kBlock, 0, s>>>(
            (const float*)fin, (float*)fout, force, d.nx, d.ny, tau0, smag, mu);
    else
        stream_collide_kernel<double><<<grid, kBlock, 0, s>>>(
            (const double*)fin, (double*)fout, force, d.nx, d.ny, tau0, smag, mu);
    return hipGetLastError();
}

hipError_t launch_import(const double* canon, void* f, LbmDims d, int storage, hipStream_t s) {
    size_t total = (size_t)d.nx * d.ny * 9 * d.members;
    if (storage == kStoreF32Dev)
        import_kernel<float><<<grid_for(total, 256), 256, 0, s>>>(canon, (float*)f, d.nx, d.ny,
                                                                  d.members);
    else
        import_kernel<double><<<grid_for(total, 256), 256, 0, s>>>(canon, (double*)f, d.nx, d.ny,
                                                                   d.members);
    return hipGetLastError();
}

hipError_t launch_export(const void* f, double* canon, LbmDims d, int storage, hipStream_t s) {
    size_t total = (size_t)d.nx * d.ny * 9 * d.members;
    if (storage == kStoreF32Dev)
        export_kernel<float><<<grid_for(total, 256), 256, 0, s>>>((const float*)f, canon, d.nx,
                                                                  d.ny, d.members);
    else
        export_kernel<double><<<grid_for(total, 256), 256, 0, s>>>((const double*)f, canon, d.nx,
                                                                   d.ny, d.members);
    return hipGetLastError();
}

hipError_t launch_init_equilibrium(const double* rho, const double* uv, void* f, LbmDims d,
                                   int storage, hipStream_t s) {
    size_t total = (size_t)d.nx * d.ny * d.members;
    if (storage == kStoreF32Dev)
        init_equilibrium_kernel<float><<<grid_for(total, 256), 256, 0, s>>>(
            rho, uv, (float*)f, d.nx, d.ny, d.members);
    else
        init_equilibrium_kernel<double><<<grid_for(total, 256), 256, 0, s>>>(
            rho, uv, (double*)f, d.nx, d.ny, d.members);
    return hipGetLastError();
}

hipError_t launch_moments(const void* f, double* out, LbmDims d, int storage, hipStream_t s) {
    size_t total = (size_t)d.nx * d.ny * d.members;
    if (storage == kStoreF32Dev)
        moments_kernel<float><<<grid_for(total, 256), 256, 0, s>>>((const float*)f, out, d.nx,
                                                                   d.ny, d.members);
    else
        moments_kernel<double><<<grid_for(total, 256), 256, 0, s>>>((const double*)f, out, d.nx,
                                                                    d.ny, d.members);
    return hipGetLastError();
}

}  // namespace lbmletkf
