// Energy spectrum of an ensemble (Sec. 4.1 shell definition; the ensemble's
// spectrum is the mean of the members' spectra, Sec. 4.3.2):
//   E(k) = M^-1 sum_m sum_{k - 1/2 <= |k'| < k + 1/2} (|u_hat_m(k')|^2 + |v_hat_m(k')|^2) / 2,
//   u_hat(k') = n^-2 sum_xi u(xi) exp(-2 pi i k'.xi / n),  u = j / rho per member.
// The 2D transform is done as two passes of direct DFT sums (no FFT): along
// x for kx = 0 .. n/2 (the velocity is real, so u_hat(-k') = conj u_hat(k')
// and the other half-plane only doubles the weight of 0 < kx < n/2), then
// along y for every ky; the mode energies are summed over the members in
// member order, then over each shell in a fixed order (deterministic).
// Off the hot path: called at report times.  Scratch comes from the
// context's ping-pong buffer.
#include "common.h"

namespace lbmletkf {
namespace {

constexpr int kSpecBlock = 256;
constexpr int kColBlock = 64;

// twiddles exp(-2 pi i j / n), j < n
__device__ __forceinline__ double2 twiddle(int j, int n) {
    double s, c;
    sincospi(2.0 * (double)j / (double)n, &s, &c);
    return make_double2(c, -s);
}

// Row pass: block (y, m).  out[(m * n + y) * ncol + kx] = (Au.re, Au.im, Av.re, Av.im),
// A(y, kx) = sum_x u(x, y) exp(-2 pi i kx x / n).
template <typename T>
__global__ __launch_bounds__(kSpecBlock) void spectrum_rows_kernel(const T* __restrict__ f, int n,
                                                                   int members,
                                                                   double4* __restrict__ out) {
    extern __shared__ double lds[];
    double* us = lds;             // [n]
    double* vs = us + n;          // [n]
    double2* tw = reinterpret_cast<double2*>(vs + n);  // [n]
    const int y = blockIdx.x, m = blockIdx.y;
    const int ncol = n / 2 + 1;
    for (int x = threadIdx.x; x < n; x += kSpecBlock) {
        double rho = 0.0, jx = 0.0, jy = 0.0;
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            const double fa = PopIO<T>::load(f + slot(src_node(x, y, a, n, n), a, m, members), a);
            rho += fa;
            jx += cx_of(a) * fa;
            jy += cy_of(a) * fa;
        }
        us[x] = jx / rho;
        vs[x] = jy / rho;
        tw[x] = twiddle(x, n);
    }
    __syncthreads();
    for (int kx = threadIdx.x; kx < ncol; kx += kSpecBlock) {
        double ur = 0.0, ui = 0.0, vr = 0.0, vi = 0.0;
        int p = 0;  // kx * x mod n
        for (int x = 0; x < n; ++x) {
            const double2 w = tw[p];
            ur += us[x] * w.x;
            ui += us[x] * w.y;
            vr += vs[x] * w.x;
            vi += vs[x] * w.y;
            p += kx;
            if (p >= n) p -= n;
        }
        out[((size_t)m * n + y) * ncol + kx] = make_double4(ur, ui, vr, vi);
    }
}

// Column pass: block (kx, ky tile).  e[ky * ncol + kx] = sum_m (|U(ky, kx)|^2 +
// |V(ky, kx)|^2) / 2 with U(ky, kx) = sum_y A(y, kx) exp(-2 pi i ky y / n),
// members summed in order.
__global__ __launch_bounds__(kColBlock) void spectrum_cols_kernel(const double4* __restrict__ rows,
                                                                  int n, int members,
                                                                  double* __restrict__ e) {
    extern __shared__ double lds[];
    double4* col = reinterpret_cast<double4*>(lds);       // [n]
    double2* tw = reinterpret_cast<double2*>(col + n);    // [n]
    const int kx = blockIdx.x;
    const int ncol = n / 2 + 1;
    const int ky = blockIdx.y * kColBlock + threadIdx.x;
    for (int j = threadIdx.x; j < n; j += kColBlock) tw[j] = twiddle(j, n);
    double acc = 0.0;
    for (int m = 0; m < members; ++m) {
        __syncthreads();
        for (int y = threadIdx.x; y < n; y += kColBlock)
            col[y] = rows[((size_t)m * n + y) * ncol + kx];
        __syncthreads();
        if (ky < n) {
            double ur = 0.0, ui = 0.0, vr = 0.0, vi = 0.0;
            int p = 0;  // ky * y mod n
            for (int y = 0; y < n; ++y) {
                const double2 w = tw[p];
                const double4 c = col[y];
                ur += c.x * w.x - c.y * w.y;
                ui += c.x * w.y + c.y * w.x;
                vr += c.z * w.x - c.w * w.y;
                vi += c.z * w.y + c.w * w.x;
                p += ky;
                if (p >= n) p -= n;
            }
            acc += 0.5 * (ur * ur + ui * ui + vr * vr + vi * vi);
        }
    }
    if (ky < n) e[(size_t)ky * ncol + kx] = acc;
}

// Shell pass: block k.  E[k] = sum over the modes of shell k (half-plane
// kx >= 0, weight 2 for 0 < kx < n/2) of e, / (M n^4), summed in a fixed order.
__global__ __launch_bounds__(kSpecBlock) void spectrum_shell_kernel(const double* __restrict__ e,
                                                                    int n, int members,
                                                                    double* __restrict__ E) {
    __shared__ double red[kSpecBlock];
    const int k = blockIdx.x;
    const int ncol = n / 2 + 1;
    const int modes = n * ncol;
    double acc = 0.0;
    for (int i = threadIdx.x; i < modes; i += kSpecBlock) {
        const int ky = i / ncol, kx = i - ky * ncol;
        const int kys = 2 * ky > n ? ky - n : ky;
        const int shell = (int)floor(sqrt((double)(kx * kx + kys * kys)) + 0.5);
        if (shell != k) continue;
        const double w = (kx == 0 || 2 * kx == n) ? 1.0 : 2.0;
        acc += w * e[i];
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kSpecBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double n2 = (double)n * (double)n;
        E[k] = red[0] / ((double)members * n2 * n2);
    }
}

template <typename K>
hipError_t allow_spec_lds(K kernel, size_t bytes) {
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
}

}  // namespace

size_t spectrum_scratch_bytes(int n, int members) {
    const size_t ncol = (size_t)n / 2 + 1;
    const size_t rows = (size_t)members * n * ncol * sizeof(double4);
    return rows + (size_t)n * ncol * sizeof(double) + 256;
}

hipError_t launch_energy_spectrum(const void* f, int n, int members, int storage, int kmax,
                                  void* scratch, double* E, hipStream_t s) {
    const size_t ncol = (size_t)n / 2 + 1;
    double4* rows = reinterpret_cast<double4*>(scratch);
    const size_t rows_bytes = (size_t)members * n * ncol * sizeof(double4);
    double* e = reinterpret_cast<double*>(reinterpret_cast<char*>(scratch) +
                                          (rows_bytes + 255) / 256 * 256);
    const size_t row_lds = (size_t)n * 4 * sizeof(double);
    hipError_t err;
    if (storage == kStoreF32Dev) {
        if ((err = allow_spec_lds(spectrum_rows_kernel<float>, row_lds)) != hipSuccess) return err;
        spectrum_rows_kernel<float><<<dim3(n, members), kSpecBlock, row_lds, s>>>(
            (const float*)f, n, members, rows);
    } else {
        if ((err = allow_spec_lds(spectrum_rows_kernel<double>, row_lds)) != hipSuccess) return err;
        spectrum_rows_kernel<double><<<dim3(n, members), kSpecBlock, row_lds, s>>>(
            (const double*)f, n, members, rows);
    }
    if ((err = hipGetLastError()) != hipSuccess) return err;
    const size_t col_lds = (size_t)n * (sizeof(double4) + sizeof(double2));
    if ((err = allow_spec_lds(spectrum_cols_kernel, col_lds)) != hipSuccess) return err;
    spectrum_cols_kernel<<<dim3((unsigned)ncol, (n + kColBlock - 1) / kColBlock), kColBlock, col_lds,
                           s>>>(rows, n, members, e);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    spectrum_shell_kernel<<<kmax + 1, kSpecBlock, 0, s>>>(e, n, members, E);
    return hipGetLastError();
}

}  // namespace lbmletkf
