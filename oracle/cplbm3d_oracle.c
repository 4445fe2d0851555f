/*
 * Plain FP64 CPU oracle of the chemical-potential lattice Boltzmann method in
 * three dimensions, D3Q19 (Wen, Zhou, He, Zhang, Fang, arXiv:1611.00907, whose
 * Sec. II states the method for any velocity set and notes that the
 * chemical-potential force saves the memory of the pressure tensor in 3-D).
 *
 * TEST INFRASTRUCTURE ONLY: the slow, obviously correct reference the GPU
 * library's 3-D step is checked against.  It shares no code, header or table
 * with the GPU library (nor with the 2-D oracle beyond restating the same
 * equations).
 *
 * One step, IEEE double, plain loops, the order of the 2-D oracle:
 *   moments -> mu = psi'(rho) - kappa lap(rho) (Eq 8; bulk terms of Eqs 18, 21,
 *   24, 27) -> F = -rho grad(mu) + c_s^2 grad(rho) (Eq 12) -> BGK collision with
 *   the equilibrium (Eq 14 on D3Q19) at u + tau F / rho -> streaming.
 * The box is periodic in x, y and z.  Readings: D3Q19 with w = 1/3 (rest),
 * 1/18 (axis), 1/36 (edge), c_s^2 = 1/3; stencils from the same weights,
 * lap = 6 sum_i w_i (phi_i - phi_0), grad = 3 sum_i w_i e_i phi_i.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { O3_VDW = 0, O3_CS = 1, O3_PR = 2, O3_RKS = 3, O3_RK = 4 };

typedef struct {
    int32_t nx, ny, nz, eos;
    double a, b, R, T, alpha;   /* EOS constants, absolute temperature, alpha(T) */
    double tau, kappa;
} o3_params;

/* D3Q19: rest, six axis directions, twelve edge directions; opposite pairs are
 * adjacent (1-2, 3-4, ...). */
static const int EX[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int EY[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int EZ[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

static double weight(int i) { return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0); }

void o3_velocities(int* ex, int* ey, int* ez, double* w) {
    for (int i = 0; i < 19; ++i) {
        ex[i] = EX[i];
        ey[i] = EY[i];
        ez[i] = EZ[i];
        w[i] = weight(i);
    }
}

/* Bulk chemical potential psi'(rho) (Eqs 18, 21, 24, 27 without the gradient term). */
static double mu_bulk(const o3_params* p, double rho) {
    const double RT = p->R * p->T, b = p->b;
    switch (p->eos) {
    case O3_VDW:
        return RT * (log(rho / (1.0 - b * rho)) + 1.0 / (1.0 - b * rho)) - 2.0 * p->a * rho;
    case O3_CS: {
        const double q = b * rho / 4.0;
        return RT * ((3.0 - q) / ((1.0 - q) * (1.0 - q) * (1.0 - q)) + log(rho) + 1.0) - 2.0 * p->a * rho;
    }
    case O3_PR: {
        const double aa = p->a * p->alpha, s2 = sqrt(2.0);
        return RT * log(rho / (1.0 - b * rho)) - aa / (2.0 * s2 * b) * log((s2 - 1.0 + b * rho) / (s2 + 1.0 - b * rho))
             + RT / (1.0 - b * rho) - aa * rho / (1.0 + 2.0 * b * rho - b * b * rho * rho);
    }
    default: { /* RK, RKS */
        const double aa = p->a * p->alpha;
        return RT * log(rho / (1.0 - b * rho)) + RT / (1.0 - b * rho) - aa / b * log(1.0 + b * rho)
             - aa * rho / (1.0 + b * rho);
    }
    }
}

static int wrap(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

static size_t idx(const o3_params* p, int x, int y, int z) {
    return ((size_t)wrap(z, p->nz) * p->ny + wrap(y, p->ny)) * p->nx + wrap(x, p->nx);
}

/* Equilibrium of Eq 14 on D3Q19. */
void o3_feq(double rho, double ux, double uy, double uz, double* feq) {
    const double usq = ux * ux + uy * uy + uz * uz;
    for (int i = 0; i < 19; ++i) {
        const double eu = EX[i] * ux + EY[i] * uy + EZ[i] * uz;
        feq[i] = rho * weight(i) * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * usq);
    }
}

static double lap19(const o3_params* p, const double* phi, int x, int y, int z) {
    const double c = phi[idx(p, x, y, z)];
    double s = 0.0;
    for (int i = 1; i < 19; ++i) s += weight(i) * (phi[idx(p, x + EX[i], y + EY[i], z + EZ[i])] - c);
    return 6.0 * s;
}

static void grad19(const o3_params* p, const double* phi, int x, int y, int z, double* g) {
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (int i = 1; i < 19; ++i) {
        const double v = weight(i) * phi[idx(p, x + EX[i], y + EY[i], z + EZ[i])];
        sx += EX[i] * v;
        sy += EY[i] * v;
        sz += EZ[i] * v;
    }
    g[0] = 3.0 * sx;
    g[1] = 3.0 * sy;
    g[2] = 3.0 * sz;
}

/* Stencil probe for the tests: Laplacian and gradient of phi. */
void o3_stencils(const o3_params* p, const double* phi, double* lap, double* gx, double* gy, double* gz) {
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                const size_t c = idx(p, x, y, z);
                double g[3];
                lap[c] = lap19(p, phi, x, y, z);
                grad19(p, phi, x, y, z, g);
                gx[c] = g[0];
                gy[c] = g[1];
                gz[c] = g[2];
            }
}

/* rho, u, mu, F of the state f (work: 9 planes). */
static void macro3(const o3_params* p, const double* f, double* w) {
    const size_t n = (size_t)p->nx * p->ny * p->nz;
    double *rho = w, *ux = w + n, *uy = w + 2 * n, *uz = w + 3 * n, *mu = w + 4 * n;
    double *Fx = w + 5 * n, *Fy = w + 6 * n, *Fz = w + 7 * n;
#pragma omp parallel for schedule(static)
    for (long long c = 0; c < (long long)n; ++c) {
        double r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
        for (int i = 0; i < 19; ++i) {
            const double v = f[i * n + c];
            r += v;
            jx += EX[i] * v;
            jy += EY[i] * v;
            jz += EZ[i] * v;
        }
        rho[c] = r;
        ux[c] = jx / r;
        uy[c] = jy / r;
        uz[c] = jz / r;
    }
#pragma omp parallel for schedule(static)
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                const size_t c = idx(p, x, y, z);
                mu[c] = mu_bulk(p, rho[c]) - p->kappa * lap19(p, rho, x, y, z);
            }
#pragma omp parallel for schedule(static)
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                const size_t c = idx(p, x, y, z);
                double gm[3], gr[3];
                grad19(p, mu, x, y, z, gm);
                grad19(p, rho, x, y, z, gr);
                Fx[c] = -rho[c] * gm[0] + gr[0] / 3.0;
                Fy[c] = -rho[c] * gm[1] + gr[1] / 3.0;
                Fz[c] = -rho[c] * gm[2] + gr[2] / 3.0;
            }
}

void o3_init(const o3_params* p, const double* rho0, double* f) {
    const size_t n = (size_t)p->nx * p->ny * p->nz;
    for (size_t c = 0; c < n; ++c) {
        double feq[19];
        o3_feq(rho0[c], 0.0, 0.0, 0.0, feq);
        for (int i = 0; i < 19; ++i) f[i * n + c] = feq[i];
    }
}

/* One step f(t) -> fnew(t+1); work holds 9 planes (rho, u, mu, F of time t on return). */
void o3_step(const o3_params* p, const double* f, double* fnew, double* work) {
    const size_t n = (size_t)p->nx * p->ny * p->nz;
    macro3(p, f, work);
    const double *rho = work, *ux = work + n, *uy = work + 2 * n, *uz = work + 3 * n;
    const double *Fx = work + 5 * n, *Fy = work + 6 * n, *Fz = work + 7 * n;
    const double tau = p->tau;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                const size_t c = idx(p, x, y, z);
                const double r = rho[c];
                double feq[19];
                o3_feq(r, ux[c] + tau * Fx[c] / r, uy[c] + tau * Fy[c] / r, uz[c] + tau * Fz[c] / r, feq);
                for (int i = 0; i < 19; ++i) {
                    const double fs = f[i * n + c] - (f[i * n + c] - feq[i]) / tau;
                    fnew[i * n + idx(p, x + EX[i], y + EY[i], z + EZ[i])] = fs;
                }
            }
}

void o3_run(const o3_params* p, double* f, double* fbuf, double* work, int64_t steps) {
    const size_t n = (size_t)19 * p->nx * p->ny * p->nz;
    for (int64_t s = 0; s < steps; ++s) {
        o3_step(p, f, fbuf, work);
        memcpy(f, fbuf, n * sizeof(double));
    }
}

/* Output fields: rho, physical velocity v = u + F / (2 rho), mu, F. */
void o3_fields(const o3_params* p, const double* f, double* work, double* rho, double* vx, double* vy, double* vz,
               double* mu, double* Fx, double* Fy, double* Fz) {
    const size_t n = (size_t)p->nx * p->ny * p->nz;
    macro3(p, f, work);
    for (size_t c = 0; c < n; ++c) {
        const double r = work[c];
        rho[c] = r;
        vx[c] = work[n + c] + work[5 * n + c] / (2.0 * r);
        vy[c] = work[2 * n + c] + work[6 * n + c] / (2.0 * r);
        vz[c] = work[3 * n + c] + work[7 * n + c] / (2.0 * r);
        mu[c] = work[4 * n + c];
        Fx[c] = work[5 * n + c];
        Fy[c] = work[6 * n + c];
        Fz[c] = work[7 * n + c];
    }
}

double o3_mass(const o3_params* p, const double* f) {
    const size_t n = (size_t)19 * p->nx * p->ny * p->nz;
    double m = 0.0;
    for (size_t k = 0; k < n; ++k) m += f[k];
    return m;
}
