// Forecast kernels: the D2Q9 lattice Boltzmann equation with BGK relaxation,
// Smagorinsky eddy viscosity and a body force (Sec. 2), advanced for every
// ensemble member in one launch (one step, or two steps on spatial tiles).
//
// Layout: f[node][a][member], node = y * nx + x, members fastest (FP64, or
// FP32 deviations).  One thread per (node, member), a block of
// (members x nodes) threads.  The kernels pull: the thread of node (x, y)
// gathers f_a from the slot of node (x - c_ax, y - c_ay), which holds the
// pre-collision population f_a(x, y, t), collides, and writes f*_a to its own
// slot (node, a).  Between steps a buffer therefore holds post-collision
// values, and the canonical f_a(x, y) lives at the slot of node
// (x - c_ax, y - c_ay); import/export convert.  With 64 members every load
// and store of a wavefront is 512 contiguous, aligned bytes.
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

// c_a . (x, y) for the D2Q9 velocity a (a constant after unrolling) as the one
// addition or sign change it needs: a multiplication by 0 or +-1 would cost an
// instruction and, without fast-math, is not dropped by the compiler.
__device__ __forceinline__ double cdot(int a, double x, double y) {
    const int cx = cx_of(a), cy = cy_of(a);
    const double tx = cx > 0 ? x : (cx < 0 ? -x : 0.0);
    if (cy == 0) return tx;
    if (cx == 0) return cy > 0 ? y : -y;
    return cy > 0 ? tx + y : tx - y;
}

// Relax one node: f[9] in (pre-collision), f*[9] out.  The multiply-adds are
// written out as fma() and the compiler may fuse nothing else, so the result
// does not depend on the code the function is inlined into: the one-step and
// the two-step kernels give the same bits.
__device__ __forceinline__ void collide_node(double (&f)[9], double tau0, double smag,
                                             double fx_ext, double fy_ext, double mu) {
#pragma clang fp contract(off)
    const double rho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
    const double jx = (f[1] - f[2]) + (f[5] - f[6]) + (f[7] - f[8]);
    const double jy = (f[3] - f[4]) + (f[5] - f[6]) + (f[8] - f[7]);
    const double inv_rho = 1.0 / rho;
    const double u = jx * inv_rho, v = jy * inv_rho;
    const double uu = u * u, vv = v * v, uv = u * v;
    // non-equilibrium momentum flux: sum c c f - rho/3 I - rho u u
    const double pxx = fma(-rho, 1.0 / 3.0 + uu, f[1] + f[2] + f[5] + f[6] + f[7] + f[8]);
    const double pyy = fma(-rho, 1.0 / 3.0 + vv, f[3] + f[4] + f[5] + f[6] + f[7] + f[8]);
    const double pxy = fma(-rho, uv, f[5] + f[6] - f[7] - f[8]);
    const double pn = sqrt(fma(pxx, pxx, fma(pyy, pyy, (2.0 * pxy) * pxy)));
    const double tau = 0.5 * (tau0 + sqrt(fma(tau0, tau0, (smag * pn) * inv_rho)));
    const double omega = 1.0 / tau;
    // acceleration: external field plus linear friction
    const double gx = fma(-mu, u, fx_ext), gy = fma(-mu, v, fy_ext);
    const double one_usq = 1.0 - 1.5 * (uu + vv);
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const double cu = cdot(a, u, v);
        // f^eq = rho w (1 + 3 cu + 4.5 cu^2 - 1.5 u.u)
        const double feq = (rho * w_of(a)) * fma(cu, fma(4.5, cu, 3.0), one_usq);
        const double Fa = (3.0 * w_of(a) * rho) * cdot(a, gx, gy);
        f[a] = fma(-omega, f[a] - feq, f[a] + Fa);
    }
}

// The same relaxation in FP32 on the deviations g_a = f_a - w_a that FP32
// storage keeps (the precision form): the lattice sums of the weights are
// exact constants (sum w = 1, sum w c = 0, sum w c c = I/3), so every moment
// is a sum of small numbers, rho = 1 + sum g,
//   Pi_xx = sum c_x^2 g - (rho - 1)/3 - rho u^2,  Pi_xy = sum c_x c_y g - rho u v,
//   g^eq_a = w_a [(rho - 1) + rho (3 cu + 4.5 cu^2 - 1.5 u.u)],
// and FP32 keeps ~7 significant digits of quantities of size |g| <~ 0.02.
__device__ __forceinline__ float cdotf(int a, float x, float y) {
    const int cx = cx_of(a), cy = cy_of(a);
    const float tx = cx > 0 ? x : (cx < 0 ? -x : 0.0f);
    if (cy == 0) return tx;
    if (cx == 0) return cy > 0 ? y : -y;
    return cy > 0 ? tx + y : tx - y;
}

__device__ __forceinline__ void collide_node_dev(float (&g)[9], float tau0, float smag,
                                                 float fx_ext, float fy_ext, float mu) {
#pragma clang fp contract(off)
    const float drho = ((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7])) + g[8];
    const float rho = 1.0f + drho;
    const float jx = (g[1] - g[2]) + (g[5] - g[6]) + (g[7] - g[8]);
    const float jy = (g[3] - g[4]) + (g[5] - g[6]) + (g[8] - g[7]);
    // 1 / rho: the hardware reciprocal (1 ulp) refined by one Newton step, three
    // instructions instead of the correctly rounded division's ten (the bare
    // reciprocal biases u enough to move a 200-step misfit by 4e-6 relative);
    // the square roots below are the hardware ones (|Pi| and R only need their
    // own relative accuracy)
    float inv_rho = __builtin_amdgcn_rcpf(rho);
    inv_rho = fmaf(inv_rho, fmaf(-rho, inv_rho, 1.0f), inv_rho);
    const float u = jx * inv_rho, v = jy * inv_rho;
    const float uu = u * u, vv = v * v, uv = u * v;
    const float d3 = drho * (1.0f / 3.0f);
    const float pxx = fmaf(-rho, uu, (g[1] + g[2] + g[5] + g[6] + g[7] + g[8]) - d3);
    const float pyy = fmaf(-rho, vv, (g[3] + g[4] + g[5] + g[6] + g[7] + g[8]) - d3);
    const float pxy = fmaf(-rho, uv, g[5] + g[6] - g[7] - g[8]);
    const float pn = __builtin_amdgcn_sqrtf(fmaf(pxx, pxx, fmaf(pyy, pyy, (2.0f * pxy) * pxy)));
    // omega = 1 / tau = 2 / (tau0 + R), R = sqrt(tau0^2 + x), x = 18 sqrt(2) C_s^2 |Pi| / rho,
    // taken as the molecular 1 / tau0 minus the eddy part x / (tau0 (tau0 + R)^2),
    // which FP32 then carries to its own relative accuracy (as 1 / tau the eddy
    // part, often 1e-4 of omega, would keep only a few bits)
    const float x = (smag * pn) * inv_rho;
    const float tr = tau0 + __builtin_amdgcn_sqrtf(fmaf(tau0, tau0, x));
    const float omega = 1.0f / tau0 - x * __builtin_amdgcn_rcpf(tau0 * tr * tr);
    const float gx = fmaf(-mu, u, fx_ext), gy = fmaf(-mu, v, fy_ext);
    const float usq = -1.5f * (uu + vv);
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const float w = (float)w_of(a);
        const float cu = cdotf(a, u, v);
        const float geq = w * fmaf(rho, fmaf(cu, fmaf(4.5f, cu, 3.0f), usq), drho);
        const float Fa = (3.0f * w * rho) * cdotf(a, gx, gy);
        g[a] = fmaf(-omega, g[a] - geq, g[a] + Fa);
    }
}

// V consecutive members per thread: FP32 deviations move 4 bytes per member,
// and one 8-byte access per population for two members keeps the wavefront's
// requests as wide as in FP64.
typedef float float2v __attribute__((ext_vector_type(2)));

// Pull, collide and store one node for members m .. m + V - 1.
template <typename T, int V>
__device__ __forceinline__ void lbm_update(const T* __restrict__ fin, T* __restrict__ fout,
                                           const double* __restrict__ force, int nx, int ny,
                                           int members, int node, int m, double tau0,
                                           double smag, double mu) {
    static_assert(V == 1 || (V == 2 && sizeof(T) == 4), "two members per thread: FP32 only");
    const int plane = nx * ny;
    const int y = node / nx, x = node - y * nx;
    const int xm = wrap_dec(x, nx), xp = wrap_inc(x, nx);
    const int ym = wrap_dec(y, ny), yp = wrap_inc(y, ny);
    // slots holding the canonical f_a(x, y): node (x - c_ax, y - c_ay)
    const PullSlots<const T> src(fin, x, xm, xp, y, ym, yp, nx, members, m);
    T* const dst = fout + (size_t)node * 9 * members + m;
    double fx = 0.0, fy = 0.0;
    if (force) {
        fx = force[node];
        fy = force[plane + node];
    }
    // every population is read once and written once per step: stream it
    // past the caches (nontemporal loads and stores)
    if constexpr (sizeof(T) == 8) {
        double f[9];
#pragma unroll
        for (int a = 0; a < 9; ++a) f[a] = PopIO<T>::load_nt(src.at(a), a);
        collide_node(f, tau0, smag, fx, fy, mu);
#pragma unroll
        for (int a = 0; a < 9; ++a) PopIO<T>::store_nt(dst + (uint32_t)a * members, a, f[a]);
    } else {
        // FP32 deviations: the FP32 relaxation on g = f - w, no conversion
        float g[V][9];
        if constexpr (V == 1) {
#pragma unroll
            for (int a = 0; a < 9; ++a)
                g[0][a] = __builtin_nontemporal_load(src.at(a));
        } else {
#pragma unroll
            for (int a = 0; a < 9; ++a) {
                const float2v p = __builtin_nontemporal_load(
                    reinterpret_cast<const float2v*>(src.at(a)));
                g[0][a] = p.x;
                g[1][a] = p.y;
            }
        }
#pragma unroll
        for (int k = 0; k < V; ++k)
            collide_node_dev(g[k], (float)tau0, (float)smag, (float)fx, (float)fy, (float)mu);
        if constexpr (V == 1) {
#pragma unroll
            for (int a = 0; a < 9; ++a)
                __builtin_nontemporal_store(g[0][a], dst + (uint32_t)a * members);
        } else {
#pragma unroll
            for (int a = 0; a < 9; ++a) {
                float2v p;
                p.x = g[0][a];
                p.y = g[1][a];
                __builtin_nontemporal_store(p, reinterpret_cast<float2v*>(dst + (uint32_t)a * members));
            }
        }
    }
}

// Members per thread of the forecast kernels: 2 for FP32 storage with an even
// ensemble, else 1 (the single and the batched step use the same choice, so
// they round identically).
__host__ __device__ constexpr int members_per_thread(int elem_bytes, int members) {
    return (elem_bytes == 4 && members % 2 == 0) ? 2 : 1;
}

template <typename T, int V>
__global__ __launch_bounds__(kBlock) void stream_collide_kernel(
    const T* __restrict__ fin, T* __restrict__ fout, const double* __restrict__ force, int nx,
    int ny, int members, double tau0, double smag, double mu) {
    const int node = blockIdx.x * blockDim.y + threadIdx.y;
    if (node >= nx * ny) return;
    lbm_update<T, V>(fin, fout, force, nx, ny, members, node, threadIdx.x * V, tau0, smag, mu);
}

// Many problems in one persistent launch: blocks of 256 threads walk the
// concatenated tile list (problem k owns tiles [tile0_k, tile0_{k+1})); a
// tile is `tile_nodes` consecutive nodes of one problem, processed as rows of
// (256 / M) nodes x M members.  The schedule is static (block b takes tiles
// b, b + gridDim.x, ...), so every launch does the same work in the same order.
template <typename T>
__global__ __launch_bounds__(kBlock) void stream_collide_batch_kernel(const LbmTask* __restrict__ tasks,
                                                                      int ntasks, int ntiles) {
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        int k = 0;
        while (k + 1 < ntasks && tasks[k + 1].tile0 <= t) ++k;
        const LbmTask& tk = tasks[k];
        const int M = tk.members;
        const int V = members_per_thread((int)sizeof(T), M);
        const int tpn = M / V;  // threads per node
        const int npb = kBlock / tpn;
        const int plane = tk.nx * tk.ny;
        const int node0 = (t - tk.tile0) * tk.tile_nodes;
        const int m = (threadIdx.x % tpn) * V, nl = threadIdx.x / tpn;
        if (nl >= npb) continue;
        for (int r = nl; r < tk.tile_nodes; r += npb) {
            const int node = node0 + r;
            if (node >= plane) break;
            if (V == 2)
                lbm_update<T, members_per_thread((int)sizeof(T), 2)>(
                    static_cast<const T*>(tk.fin), static_cast<T*>(tk.fout), tk.force, tk.nx,
                    tk.ny, M, node, m, tk.tau0, tk.smag, tk.mu);
            else
                lbm_update<T, 1>(static_cast<const T*>(tk.fin), static_cast<T*>(tk.fout), tk.force,
                                 tk.nx, tk.ny, M, node, m, tk.tau0, tk.smag, tk.mu);
        }
    }
}

// Two steps per launch on spatial tiles.  A block takes kTwoMG members of a
// kTwoT x kTwoT tile of nodes: its first step covers the tile and a one-node
// ring around it (kTwoR x kTwoR nodes, one thread per node and member, exactly
// the single step's arithmetic on the same inputs) and keeps the results in
// LDS, rounded as a store and reload would round them; its second step pulls
// from there for the tile's nodes and writes them.  HBM traffic per two steps
// is kTwoR^2 / kTwoT^2 reads plus one write of the tile instead of two reads
// and two writes (0.69x for 6 x 6 tiles).
constexpr int kTwoMG = 16;
constexpr int kTwoT = 6;
constexpr int kTwoR = kTwoT + 2;

__host__ __device__ constexpr int two_step_lds_doubles() { return kTwoR * kTwoR * 9 * kTwoMG; }

// Block b of a two-step launch over one problem (FP64 storage): member group
// b % (members / kTwoMG) of tile b / (members / kTwoMG).
__device__ __forceinline__ void two_step_body(const double* __restrict__ fin,
                                              double* __restrict__ fout,
                                              const double* __restrict__ force, int nx, int ny,
                                              int members, double tau0, double smag, double mu,
                                              int b, double* __restrict__ fmid) {
    extern __shared__ double mid[];  // [kTwoR * kTwoR][9][kTwoMG]
    using T = double;
    const int groups = members / kTwoMG;
    const int tiles_x = (nx + kTwoT - 1) / kTwoT;
    const int mg = b % groups, tile = b / groups;
    const int x0 = (tile % tiles_x) * kTwoT, y0 = (tile / tiles_x) * kTwoT;
    const int m = mg * kTwoMG + threadIdx.x;
    const int r = threadIdx.y, rx = r % kTwoR, ry = r / kTwoR;
    // this thread's region node, periodic (a ragged edge tile computes a few
    // nodes nobody reads)
    const int gx = (x0 - 1 + rx + nx) % nx, gy = (y0 - 1 + ry + ny) % ny;
    const int plane = nx * ny;
    const int node = gy * nx + gx;
    double fx = 0.0, fy = 0.0;
    if (force) {
        fx = force[node];
        fy = force[plane + node];
    }
    const PullSlots<const T> src(fin, gx, wrap_dec(gx, nx), wrap_inc(gx, nx), gy, wrap_dec(gy, ny),
                                 wrap_inc(gy, ny), nx, members, m);
    const size_t own_slot = (size_t)node * 9 * members + m;
    // first step: the single step's pull and collision
    double f[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) f[a] = PopIO<T>::load_nt(src.at(a), a);
    collide_node(f, tau0, smag, fx, fy, mu);
#pragma unroll
    for (int a = 0; a < 9; ++a) mid[(r * 9 + a) * kTwoMG + threadIdx.x] = PopIO<T>::round(f[a], a);
    const int ix = rx - 1, iy = ry - 1;
    const bool own = ix >= 0 && ix < kTwoT && iy >= 0 && iy < kTwoT && x0 + ix < nx && y0 + iy < ny;
    // the first step's state of the tile's own nodes, when asked for
    if (fmid && own) {
#pragma unroll
        for (int a = 0; a < 9; ++a)
            PopIO<T>::store_nt(fmid + own_slot + (uint32_t)a * members, a, f[a]);
    }
    __syncthreads();
    // second step for the tile's own nodes
    if (!own) return;
#pragma unroll
    for (int a = 0; a < 9; ++a)
        f[a] = mid[(((ry - cy_of(a)) * kTwoR + rx - cx_of(a)) * 9 + a) * kTwoMG + threadIdx.x];
    collide_node(f, tau0, smag, fx, fy, mu);
#pragma unroll
    for (int a = 0; a < 9; ++a) PopIO<T>::store_nt(fout + own_slot + (uint32_t)a * members, a, f[a]);
}

__global__ __launch_bounds__(kTwoMG * kTwoR * kTwoR) void stream_collide2_kernel(
    const double* __restrict__ fin, double* __restrict__ fout, const double* __restrict__ force,
    int nx, int ny, int members, double tau0, double smag, double mu, double* __restrict__ fmid) {
    two_step_body(fin, fout, force, nx, ny, members, tau0, smag, mu, blockIdx.x, fmid);
}

// The two-step kernel for FP32 storage: the FP32 relaxation on deviations
// (collide_node_dev), MG members per block as MG / 2 threads of two adjacent
// members each (8-byte accesses, as in the single step), the intermediate
// deviations kept in LDS as FP32 -- exactly the values a single step would
// store -- so that a launch equals two single-step launches bit for bit.
// Block b of a two-step launch over one problem (FP32 storage): member group
// b % (members / gsize) of tile b / (members / gsize), gsize <= MG members per
// group (threads with 2 threadIdx.x >= gsize idle: a batch runs 16-member
// problems in 32-member blocks).
template <int MG>
__device__ __forceinline__ void two_step_dev_body(const float* __restrict__ fin,
                                                  float* __restrict__ fout,
                                                  const double* __restrict__ force, int nx, int ny,
                                                  int members, float tau0, float smag, float mu,
                                                  int b, int gsize, float* __restrict__ fmid) {
    extern __shared__ float mids[];  // [kTwoR * kTwoR][9][MG]
    typedef float f2 __attribute__((ext_vector_type(2)));
    const int groups = members / gsize;
    const int tiles_x = (nx + kTwoT - 1) / kTwoT;
    const int mg = b % groups, tile = b / groups;
    const int x0 = (tile % tiles_x) * kTwoT, y0 = (tile / tiles_x) * kTwoT;
    const int mp = 2 * threadIdx.x;          // first member of the pair within the group
    const bool on = mp < gsize;
    const int m = mg * gsize + (on ? mp : 0);
    const int r = threadIdx.y, rx = r % kTwoR, ry = r / kTwoR;
    const int gx = (x0 - 1 + rx + nx) % nx, gy = (y0 - 1 + ry + ny) % ny;
    const int plane = nx * ny;
    const int node = gy * nx + gx;
    float fx = 0.0f, fy = 0.0f;
    if (force) {
        fx = (float)force[node];
        fy = (float)force[plane + node];
    }
    const PullSlots<const float> src(fin, gx, wrap_dec(gx, nx), wrap_inc(gx, nx), gy,
                                     wrap_dec(gy, ny), wrap_inc(gy, ny), nx, members, m);
    const size_t own_slot = (size_t)node * 9 * members + m;
    float g0[9], g1[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const f2 v = __builtin_nontemporal_load(reinterpret_cast<const f2*>(src.at(a)));
        g0[a] = v.x;
        g1[a] = v.y;
    }
    collide_node_dev(g0, tau0, smag, fx, fy, mu);
    collide_node_dev(g1, tau0, smag, fx, fy, mu);
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        f2 v;
        v.x = g0[a];
        v.y = g1[a];
        *reinterpret_cast<f2*>(mids + (r * 9 + a) * MG + mp) = v;
    }
    const int ix = rx - 1, iy = ry - 1;
    const bool own = on && ix >= 0 && ix < kTwoT && iy >= 0 && iy < kTwoT && x0 + ix < nx &&
                     y0 + iy < ny;
    // the first step's state of the tile's own nodes, when asked for
    if (fmid && own) {
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            f2 v;
            v.x = g0[a];
            v.y = g1[a];
            __builtin_nontemporal_store(
                v, reinterpret_cast<f2*>(fmid + own_slot + (uint32_t)a * members));
        }
    }
    __syncthreads();
    if (!own) return;
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const f2 v = *reinterpret_cast<const f2*>(
            mids + (((ry - cy_of(a)) * kTwoR + rx - cx_of(a)) * 9 + a) * MG + mp);
        g0[a] = v.x;
        g1[a] = v.y;
    }
    collide_node_dev(g0, tau0, smag, fx, fy, mu);
    collide_node_dev(g1, tau0, smag, fx, fy, mu);
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        f2 v;
        v.x = g0[a];
        v.y = g1[a];
        __builtin_nontemporal_store(v, reinterpret_cast<f2*>(fout + own_slot + (uint32_t)a * members));
    }
}

template <int MG>
__global__ __launch_bounds__(MG / 2 * kTwoR * kTwoR) void stream_collide2_dev_kernel(
    const float* __restrict__ fin, float* __restrict__ fout, const double* __restrict__ force,
    int nx, int ny, int members, float tau0, float smag, float mu, float* __restrict__ fmid) {
    two_step_dev_body<MG>(fin, fout, force, nx, ny, members, tau0, smag, mu, blockIdx.x, MG, fmid);
}

// Two steps of many problems in one launch: block b belongs to the task k
// with block0_k <= b < block0_{k+1} (a problem's blocks are its tiles x member
// groups: 16 members for FP64 storage, 32 -- or 16 for a 16-member problem --
// for FP32 storage), and runs that problem's two-step block b - block0_k.
constexpr int kTwoMG32 = 32;  // members per block of the FP32 batched launch

template <typename T>
__global__ __launch_bounds__((sizeof(T) == 8 ? kTwoMG : kTwoMG32 / 2) * kTwoR * kTwoR) void
stream_collide2_batch_kernel(const LbmTask* __restrict__ tasks, int ntasks) {
    const int b = blockIdx.x;
    int k = 0;
    while (k + 1 < ntasks && tasks[k + 1].block0 <= b) ++k;
    const LbmTask& tk = tasks[k];
    if constexpr (sizeof(T) == 8)
        two_step_body(static_cast<const double*>(tk.fin), static_cast<double*>(tk.fout), tk.force,
                      tk.nx, tk.ny, tk.members, tk.tau0, tk.smag, tk.mu, b - tk.block0, nullptr);
    else
        two_step_dev_body<kTwoMG32>(static_cast<const float*>(tk.fin),
                                    static_cast<float*>(tk.fout), tk.force, tk.nx, tk.ny,
                                    tk.members, (float)tk.tau0, (float)tk.smag, (float)tk.mu,
                                    b - tk.block0, tk.members % kTwoMG32 == 0 ? kTwoMG32 : kTwoMG,
                                    nullptr);
}

// storage slot (node (x, y), a, m) <- canonical [m][a][y + c_ay][x + c_ax]
template <typename T>
__global__ void import_kernel(const double* __restrict__ canon, T* __restrict__ f, int nx,
                              int ny, int members) {
    const size_t plane = (size_t)nx * ny;
    const size_t total = plane * 9 * members;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total;
         t += (size_t)gridDim.x * blockDim.x) {
        const int m = (int)(t % members);
        const size_t r = t / members;
        const int a = (int)(r % 9);
        const size_t node = r / 9;
        const int y = (int)(node / nx), x = (int)(node % nx);
        const int xs = wrap1(x + cx_of(a), nx), ys = wrap1(y + cy_of(a), ny);
        PopIO<T>::store(f + t, a, canon[((size_t)m * 9 + a) * plane + (size_t)ys * nx + xs]);
    }
}

// canonical [m][a][y][x] <- storage slot (node (x - c_ax, y - c_ay), a, m)
template <typename T>
__global__ void export_kernel(const T* __restrict__ f, double* __restrict__ canon, int nx,
                              int ny, int members) {
    const size_t plane = (size_t)nx * ny;
    const size_t total = plane * 9 * members;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total;
         t += (size_t)gridDim.x * blockDim.x) {
        const size_t i = t % plane;
        const int a = (int)((t / plane) % 9);
        const int m = (int)(t / (plane * 9));
        const int y = (int)(i / nx), x = (int)(i % nx);
        canon[t] = PopIO<T>::load(f + slot(src_node(x, y, a, nx, ny), a, m, members), a);
    }
}

// f^eq(rho, u) of node (x, y), written to the slots that hold its canonical populations.
template <typename T>
__global__ void init_equilibrium_kernel(const double* __restrict__ rho_in,
                                        const double* __restrict__ uv, T* __restrict__ f, int nx,
                                        int ny, int members) {
    const size_t plane = (size_t)nx * ny;
    const size_t total = plane * members;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total;
         t += (size_t)gridDim.x * blockDim.x) {
        const int m = (int)(t % members);
        const size_t i = t / members;
        const int y = (int)(i / nx), x = (int)(i % nx);
        const double rho = rho_in ? rho_in[(size_t)m * plane + i] : 1.0;
        const double u = uv[((size_t)m * 2) * plane + i], v = uv[((size_t)m * 2 + 1) * plane + i];
        const double usq = 1.5 * (u * u + v * v);
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            const double cu = cx_of(a) * u + cy_of(a) * v;
            PopIO<T>::store(f + slot(src_node(x, y, a, nx, ny), a, m, members), a,
                            rho * w_of(a) * (1.0 + 3.0 * cu + 4.5 * cu * cu - usq));
        }
    }
}

// rho, u, v of every node from the canonical populations: out[m][3][y][x].
template <typename T>
__global__ void moments_kernel(const T* __restrict__ f, double* __restrict__ out, int nx,
                               int ny, int members) {
    const size_t plane = (size_t)nx * ny;
    const size_t total = plane * members;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total;
         t += (size_t)gridDim.x * blockDim.x) {
        const size_t i = t % plane;
        const int m = (int)(t / plane);
        const int y = (int)(i / nx), x = (int)(i % nx);
        double rho = 0.0, jx = 0.0, jy = 0.0;
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            const double fa =
                PopIO<T>::load(f + slot(src_node(x, y, a, nx, ny), a, m, members), a);
            rho += fa;
            jx += cx_of(a) * fa;
            jy += cy_of(a) * fa;
        }
        out[((size_t)m * 3) * plane + i] = rho;
        out[((size_t)m * 3 + 1) * plane + i] = jx / rho;
        out[((size_t)m * 3 + 2) * plane + i] = jy / rho;
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
    const int V = members_per_thread((int)state_elem_bytes(storage), d.members);
    const int tpn = d.members / V;
    const int npb = nodes_per_block(tpn);
    const dim3 block(tpn, npb);
    const dim3 grid((plane + npb - 1) / npb);
    const double smag = 18.0 * sqrt(2.0) * cs * cs;
    if (storage == kStoreF32Dev && V == 2)
        stream_collide_kernel<float, 2><<<grid, block, 0, s>>>(
            (const float*)fin, (float*)fout, force, d.nx, d.ny, d.members, tau0, smag, mu);
    else if (storage == kStoreF32Dev)
        stream_collide_kernel<float, 1><<<grid, block, 0, s>>>(
            (const float*)fin, (float*)fout, force, d.nx, d.ny, d.members, tau0, smag, mu);
    else
        stream_collide_kernel<double, 1><<<grid, block, 0, s>>>(
            (const double*)fin, (double*)fout, force, d.nx, d.ny, d.members, tau0, smag, mu);
    return hipGetLastError();
}

bool two_step_supported(LbmDims d, int storage) {
    // FP64: blocks of 16 members; FP32 deviations: 32 (or 16) members as pairs
    return d.members % kTwoMG == 0;
}

hipError_t launch_stream_collide2(const void* fin, void* fout, const double* force, LbmDims d,
                                  double tau0, double cs, double mu, int storage, hipStream_t s,
                                  void* fmid) {
    if (!two_step_supported(d, storage)) return hipErrorInvalidValue;
    const int tiles = ((d.nx + kTwoT - 1) / kTwoT) * ((d.ny + kTwoT - 1) / kTwoT);
    const double smag = 18.0 * sqrt(2.0) * cs * cs;
    hipError_t e = hipSuccess;
    if (storage == kStoreF32Dev) {
        static bool attr32 = false, attr16 = false;
        if (d.members % 32 == 0) {
            const size_t bytes = (size_t)kTwoR * kTwoR * 9 * 32 * sizeof(float);
            if (!attr32)
                e = hipFuncSetAttribute(reinterpret_cast<const void*>(stream_collide2_dev_kernel<32>),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
            if (e != hipSuccess) return e;
            attr32 = true;
            stream_collide2_dev_kernel<32><<<tiles * (d.members / 32), dim3(16, kTwoR * kTwoR),
                                             bytes, s>>>((const float*)fin, (float*)fout, force,
                                                         d.nx, d.ny, d.members, (float)tau0,
                                                         (float)smag, (float)mu, (float*)fmid);
        } else {
            const size_t bytes = (size_t)kTwoR * kTwoR * 9 * 16 * sizeof(float);
            if (!attr16)
                e = hipFuncSetAttribute(reinterpret_cast<const void*>(stream_collide2_dev_kernel<16>),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
            if (e != hipSuccess) return e;
            attr16 = true;
            stream_collide2_dev_kernel<16><<<tiles * (d.members / 16), dim3(8, kTwoR * kTwoR),
                                             bytes, s>>>((const float*)fin, (float*)fout, force,
                                                         d.nx, d.ny, d.members, (float)tau0,
                                                         (float)smag, (float)mu, (float*)fmid);
        }
        return hipGetLastError();
    }
    const dim3 grid(tiles * (d.members / kTwoMG)), block(kTwoMG, kTwoR * kTwoR);
    const size_t bytes = (size_t)two_step_lds_doubles() * sizeof(double);
    static bool attr = false;
    if (!attr)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(stream_collide2_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
    attr = true;
    stream_collide2_kernel<<<grid, block, bytes, s>>>(
        (const double*)fin, (double*)fout, force, d.nx, d.ny, d.members, tau0, smag, mu,
        (double*)fmid);
    return hipGetLastError();
}

hipError_t launch_stream_collide_batch(const LbmTask* d_tasks, int ntasks, int ntiles, int blocks,
                                       int storage, hipStream_t s) {
    if (storage == kStoreF32Dev)
        stream_collide_batch_kernel<float><<<blocks, kBlock, 0, s>>>(d_tasks, ntasks, ntiles);
    else
        stream_collide_batch_kernel<double><<<blocks, kBlock, 0, s>>>(d_tasks, ntasks, ntiles);
    return hipGetLastError();
}

int two_step_blocks(LbmDims d, int storage) {
    const int g = (storage == kStoreF32Dev && d.members % kTwoMG32 == 0) ? kTwoMG32 : kTwoMG;
    return ((d.nx + kTwoT - 1) / kTwoT) * ((d.ny + kTwoT - 1) / kTwoT) * (d.members / g);
}

hipError_t launch_stream_collide2_batch(const LbmTask* d_tasks, int ntasks, int nblocks,
                                        int storage, hipStream_t s) {
    static bool attr64 = false, attr32 = false;
    hipError_t e = hipSuccess;
    if (storage == kStoreF32Dev) {
        const size_t bytes = (size_t)kTwoR * kTwoR * 9 * kTwoMG32 * sizeof(float);
        if (!attr32)
            e = hipFuncSetAttribute(reinterpret_cast<const void*>(stream_collide2_batch_kernel<float>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
        attr32 = true;
        stream_collide2_batch_kernel<float><<<nblocks, dim3(kTwoMG32 / 2, kTwoR * kTwoR), bytes,
                                              s>>>(d_tasks, ntasks);
    } else {
        const size_t bytes = (size_t)two_step_lds_doubles() * sizeof(double);
        if (!attr64)
            e = hipFuncSetAttribute(reinterpret_cast<const void*>(stream_collide2_batch_kernel<double>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
        attr64 = true;
        stream_collide2_batch_kernel<double><<<nblocks, dim3(kTwoMG, kTwoR * kTwoR), bytes, s>>>(
            d_tasks, ntasks);
    }
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
