/*
 * FP64 reference lattice-Boltzmann step -- TEST INFRASTRUCTURE ONLY.
 *
 * Part of the oracle: a plain, slow, obviously correct CPU implementation
 * that the GPU path is checked against.  Only the tests, the smoke check and
 * the benchmark's CPU-baseline leg may load it.  It shares no code with the
 * GPU library.
 *
 * What it computes (Sec. 2 of Hasegawa et al., LBM-LETKF):
 *   D2Q9 velocities c_a, weights w_a (Sec. 2, velocity set and weights);
 *   lattice Boltzmann equation with BGK relaxation and a force term,
 *     f_a(x + c_a, t + 1) = f_a(x, t) - (f_a - f_a^eq)/tau + F_a      (LBE)
 *   moments rho = sum f_a, u = sum f_a c_a / rho;
 *   equilibrium f^eq = rho w (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u);
 *   forcing F_a = 3 w_a rho (F . c_a);
 *   relaxation time from nu + nu_SGS = (tau - 1/2)/3 with the Smagorinsky
 *   viscosity nu_SGS = C_s^2 |S|, |S| = sqrt(2 S_ij S_ij), filter width dx.
 * Lattice units dx = dt = c = 1.
 *
 * Readings of what the paper leaves open:
 *   velocity order 0:(0,0) 1:(1,0) 2:(-1,0) 3:(0,1) 4:(0,-1) 5:(1,1)
 *     6:(-1,-1) 7:(1,-1) 8:(-1,1);
 *   the strain rate comes from the local non-equilibrium stress
 *     Pi_ij = sum_a c_ai c_aj (f_a - f_a^eq) through the Chapman-Enskog
 *     relation S_ij = -3 Pi_ij / (2 rho tau); with tau = tau0 + 3 C_s^2 |S|
 *     this is a quadratic in tau whose positive root is used;
 *   the acceleration is F = F_ext(x) - mu u (external field plus the linear
 *     friction of Sec. 4.1), u taken without a half-force shift;
 *   the state is the pre-collision population f(x, t) at every node, stored
 *   [member][a][y][x], x fastest, doubly periodic.
 *
 * Built with gcc -O2 -ffp-contract=off -fopenmp (parallel over rows of all members).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

static const int CX[9] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
static const int CY[9] = {0, 0, 0, 1, -1, 1, -1, -1, 1};
static const double W[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                            1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

/* Expose the lattice so tests can check its moments. */
void oracle_lattice(int* cx, int* cy, double* w) {
    for (int a = 0; a < 9; ++a) {
        cx[a] = CX[a];
        cy[a] = CY[a];
        w[a] = W[a];
    }
}

static void equilibrium9(double rho, double ux, double uy, double* feq) {
    double uu = ux * ux + uy * uy;
    for (int a = 0; a < 9; ++a) {
        double cu = CX[a] * ux + CY[a] * uy;
        feq[a] = rho * W[a] * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    }
}

/* f^eq(rho, u) at every node of every member; rho, ux, uy are [M][ny][nx]. */
void oracle_equilibrium(const double* rho, const double* ux, const double* uy,
                        double* f, int nx, int ny, int members) {
    size_t plane = (size_t)nx * ny;
    for (int m = 0; m < members; ++m)
        for (size_t i = 0; i < plane; ++i) {
            double feq[9];
            size_t k = (size_t)m * plane + i;
            equilibrium9(rho[k], ux[k], uy[k], feq);
            for (int a = 0; a < 9; ++a) f[((size_t)m * 9 + a) * plane + i] = feq[a];
        }
}

/* rho, u, v of every node: outputs [M][ny][nx]. */
void oracle_moments(const double* f, double* rho, double* ux, double* uy,
                    int nx, int ny, int members) {
    size_t plane = (size_t)nx * ny;
    for (int m = 0; m < members; ++m)
        for (size_t i = 0; i < plane; ++i) {
            double r = 0.0, jx = 0.0, jy = 0.0;
            for (int a = 0; a < 9; ++a) {
                double fa = f[((size_t)m * 9 + a) * plane + i];
                r += fa;
                jx += fa * CX[a];
                jy += fa * CY[a];
            }
            size_t k = (size_t)m * plane + i;
            rho[k] = r;
            ux[k] = jx / r;
            uy[k] = jy / r;
        }
}

/* Relaxation time of one node from its nine populations (Sec. 2, Smagorinsky). */
double oracle_relaxation_time(const double* f9, double tau0, double cs) {
    double rho = 0.0, jx = 0.0, jy = 0.0;
    for (int a = 0; a < 9; ++a) {
        rho += f9[a];
        jx += f9[a] * CX[a];
        jy += f9[a] * CY[a];
    }
    double ux = jx / rho, uy = jy / rho, feq[9];
    equilibrium9(rho, ux, uy, feq);
    double pxx = 0.0, pyy = 0.0, pxy = 0.0;
    for (int a = 0; a < 9; ++a) {
        double fneq = f9[a] - feq[a];
        pxx += CX[a] * CX[a] * fneq;
        pyy += CY[a] * CY[a] * fneq;
        pxy += CX[a] * CY[a] * fneq;
    }
    double pnorm = sqrt(pxx * pxx + pyy * pyy + 2.0 * pxy * pxy);
    return 0.5 * (tau0 + sqrt(tau0 * tau0 + 18.0 * sqrt(2.0) * cs * cs * pnorm / rho));
}

/*
 * Collide-and-stream of one lattice row y of one member: f_out(x + c_a) = f*_a(x).
 * force is [2][ny][nx] (external acceleration); may be NULL for no force.
 */
static void step_row(const double* fin, double* fout, int nx, int ny, int y, double tau0,
                     double cs, const double* force, double mu) {
    size_t plane = (size_t)nx * ny;
    for (int x = 0; x < nx; ++x) {
        size_t i = (size_t)y * nx + x;
        double f9[9], feq[9];
        double rho = 0.0, jx = 0.0, jy = 0.0;
        for (int a = 0; a < 9; ++a) {
            f9[a] = fin[(size_t)a * plane + i];
            rho += f9[a];
            jx += f9[a] * CX[a];
            jy += f9[a] * CY[a];
        }
        double ux = jx / rho, uy = jy / rho;
        equilibrium9(rho, ux, uy, feq);
        double tau = oracle_relaxation_time(f9, tau0, cs);
        double fx = -mu * ux, fy = -mu * uy;
        if (force) {
            fx += force[i];
            fy += force[plane + i];
        }
        for (int a = 0; a < 9; ++a) {
            double Fa = 3.0 * W[a] * rho * (fx * CX[a] + fy * CY[a]);
            double fstar = f9[a] - (f9[a] - feq[a]) / tau + Fa;
            int xd = (x + CX[a] + nx) % nx;
            int yd = (y + CY[a] + ny) % ny;
            fout[(size_t)a * plane + (size_t)yd * nx + xd] = fstar;
        }
    }
}

/* Advance f ([M][9][ny][nx], in place) by nsteps steps. Returns 0, or -1 on OOM. */
int oracle_lbm_steps(double* f, int nx, int ny, int members, double tau0, double cs,
                     const double* force, double mu, int nsteps) {
    size_t n = (size_t)members * 9 * nx * ny;
    double* tmp = (double*)malloc(n * sizeof(double));
    if (!tmp) return -1;
    size_t per = (size_t)9 * nx * ny;
    for (int s = 0; s < nsteps; ++s) {
#pragma omp parallel for schedule(static)
        for (long r = 0; r < (long)members * ny; ++r) {
            int m = (int)(r / ny), y = (int)(r % ny);
            step_row(f + m * per, tmp + m * per, nx, ny, y, tau0, cs, force, mu);
        }
        memcpy(f, tmp, n * sizeof(double));
    }
    free(tmp);
    return 0;
}
