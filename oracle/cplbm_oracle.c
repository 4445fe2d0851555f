/*
 * Plain FP64 CPU oracle of the chemical-potential lattice Boltzmann method
 * (Wen, Zhou, He, Zhang, Fang, "Chemical-potential-based lattice Boltzmann
 * method for nonideal fluids", arXiv:1611.00907).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product never links, imports or calls it, and it shares no code, header or
 * table with the GPU library.
 *
 * Everything is IEEE double, plain loops, one phase of the algorithm at a
 * time, in the order the paper states the method:
 *   moments (Eq 13 state, Eq 14 velocity)  ->  solid-node density (Eq 28)
 *   ->  chemical potential mu = psi'(rho) - kappa lap(rho) (Eq 8 with the
 *       bulk terms of Eqs 18, 21, 24, 27) with the wall value (Sec. IV, V)
 *   ->  nonideal force F = -rho grad(mu) + grad(c_s^2 rho) (Eq 12, P0 of Eq 5)
 *   ->  BGK collision with the equilibrium velocity u + tau F / rho (Eqs 13, 14
 *       and the forcing paragraph after Eq 14)
 *   ->  streaming, with bounce-back for links that enter a solid row (Sec. IV).
 * Two variants that Sec. II names stand beside it: the force as the divergence
 * of the full pressure tensor (Eq 5 with P from Eq 9, periodic lattices), and
 * the TRT and MRT collision operators in place of BGK.
 *
 * Readings where the paper is silent (all listed in the design notes):
 *   D2Q9 with w = 4/9, 1/9, 1/36 (the coefficients of Eq 14 give c_s^2 = 1/3);
 *   isotropic 9-point stencils lap = 6 sum_i w_i (phi_i - phi_0) and
 *   grad = 3 sum_i w_i e_i phi_i; halfway (link) bounce-back between the solid
 *   row and the first fluid row; the Eq 28 ghost density also enters the
 *   c_s^2 grad(rho) term at the first fluid row; solid rows hold no
 *   distributions.
 *
 * OpenMP parallelises each phase over rows; every cell is computed
 * independently, so results do not depend on the thread count.  The mass sum
 * is a serial loop in a fixed order.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Boundary kinds of the bottom (y = 0) and top (y = ny-1) rows. */
enum { ORA_PERIODIC = 0, ORA_CPWALL = 1, ORA_NEUTRAL = 2 };
/* Equations of state of Sec. III. */
enum { ORA_VDW = 0, ORA_CS = 1, ORA_PR = 2, ORA_RKS = 3, ORA_RK = 4 };

typedef struct {
    int32_t nx, ny;          /* lattice nodes including solid rows          */
    int32_t bottom, top;     /* ORA_PERIODIC (both) or a wall kind          */
    int32_t eos;             /* ORA_VDW ...                                 */
    int32_t scheme;          /* force (bits 0-3) | collision (bits 4-7)     */
    double a, b, R, T;       /* EOS constants and absolute temperature       */
    double alpha;            /* alpha(T) of Eqs 19/22 (1 for VdW and CS)     */
    double tau, kappa;       /* relaxation time (Eq 13), gradient coeff (Eq 1) */
    double trt_lambda;       /* TRT: (tau+ - 1/2)(tau- - 1/2)                  */
    double s_e, s_eps, s_q;  /* MRT relaxation rates of e, epsilon, q          */
} ora_params;

/* Nonideal force: the chemical-potential form of Eq 12 (the paper's method) or
 * the divergence of the pressure tensor, Eq 5 with P from Eq 9. */
enum { ORA_FORCE_CP = 0, ORA_FORCE_PTENSOR = 1 };
/* Collision (Sec. II names BGK, MRT and TRT): BGK of Eq 13; two relaxation
 * times (even part at 1/tau, odd part at 1/tau- with (tau - 1/2)(tau- - 1/2) =
 * lambda); multiple relaxation times on the D2Q9 moments of Lallemand and Luo
 * (Phys. Rev. E 61, 6546, 2000). */
enum { ORA_COLLIDE_BGK = 0, ORA_COLLIDE_TRT = 16, ORA_COLLIDE_MRT = 32 };

/* D2Q9: 0 rest, 1..4 axis, 5..8 diagonal. */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const double W[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                            1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

/* ------------------------------------------------------------------------ */
/* Equations of state: pressure p0, free-energy density psi and bulk chemical
 * potential mu_b = psi'(rho) (Eq 8 without the gradient term).               */
/* ------------------------------------------------------------------------ */

/* Van der Waals: Eqs 16, 17, 18. */
static void eos_vdw(const ora_params* p, double rho, double* psi, double* p0, double* mub) {
    const double RT = p->R * p->T, a = p->a, b = p->b;
    *p0 = rho * RT / (1.0 - b * rho) - a * rho * rho;
    *psi = rho * RT * log(rho / (1.0 - b * rho)) - a * rho * rho;
    *mub = RT * (log(rho / (1.0 - b * rho)) + 1.0 / (1.0 - b * rho)) - 2.0 * a * rho;
}

/* Redlich-Kwong and its Soave form share Eqs 19, 20, 21; only alpha(T) differs. */
static void eos_rk(const ora_params* p, double rho, double* psi, double* p0, double* mub) {
    const double RT = p->R * p->T, aa = p->a * p->alpha, b = p->b;
    *p0 = rho * RT / (1.0 - b * rho) - aa * rho * rho / (1.0 + b * rho);
    *psi = RT * rho * log(rho / (1.0 - b * rho)) - aa / b * rho * log(1.0 + b * rho);
    *mub = RT * log(rho / (1.0 - b * rho)) + RT / (1.0 - b * rho)
         - aa / b * log(1.0 + b * rho) - aa * rho / (1.0 + b * rho);
}

/* Peng-Robinson: Eqs 22, 23, 24. */
static void eos_pr(const ora_params* p, double rho, double* psi, double* p0, double* mub) {
    const double RT = p->R * p->T, aa = p->a * p->alpha, b = p->b;
    const double s2 = sqrt(2.0);
    const double den = 1.0 + 2.0 * b * rho - b * b * rho * rho;
    const double lg = log((s2 - 1.0 + b * rho) / (s2 + 1.0 - b * rho));
    *p0 = rho * RT / (1.0 - b * rho) - aa * rho * rho / den;
    *psi = RT * rho * log(rho / (1.0 - b * rho)) - aa * rho / (2.0 * s2 * b) * lg;
    *mub = RT * log(rho / (1.0 - b * rho)) - aa / (2.0 * s2 * b) * lg
         + RT / (1.0 - b * rho) - aa * rho / den;
}

/* Carnahan-Starling: Eqs 25, 26, 27. */
static void eos_cs(const ora_params* p, double rho, double* psi, double* p0, double* mub) {
    const double RT = p->R * p->T, a = p->a, b = p->b;
    const double q = b * rho / 4.0;
    *p0 = rho * RT * (1.0 + q + q * q - q * q * q) / ((1.0 - q) * (1.0 - q) * (1.0 - q)) - a * rho * rho;
    *psi = RT * rho * ((3.0 - b * rho / 2.0) / ((1.0 - q) * (1.0 - q)) + log(rho)) - a * rho * rho;
    *mub = RT * ((3.0 - q) / ((1.0 - q) * (1.0 - q) * (1.0 - q)) + log(rho) + 1.0) - 2.0 * a * rho;
}

static void eos_eval(const ora_params* p, double rho, double* psi, double* p0, double* mub) {
    switch (p->eos) {
    case ORA_VDW: eos_vdw(p, rho, psi, p0, mub); break;
    case ORA_CS: eos_cs(p, rho, psi, p0, mub); break;
    case ORA_PR: eos_pr(p, rho, psi, p0, mub); break;
    default: eos_rk(p, rho, psi, p0, mub); break; /* ORA_RKS, ORA_RK */
    }
}

/* Vectorised EOS evaluation for the Python side of the oracle. */
void ora_eos(const ora_params* p, int64_t n, const double* rho, double* psi, double* p0, double* mub) {
    for (int64_t k = 0; k < n; ++k) {
        double s, q, m;
        eos_eval(p, rho[k], &s, &q, &m);
        if (psi) psi[k] = s;
        if (p0) p0[k] = q;
        if (mub) mub[k] = m;
    }
}

/* ------------------------------------------------------------------------ */
/* Lattice helpers                                                           */
/* ------------------------------------------------------------------------ */

static int is_solid_row(const ora_params* p, int y) {
    if (p->bottom != ORA_PERIODIC && y == 0) return 1;
    if (p->top != ORA_PERIODIC && y == p->ny - 1) return 1;
    return 0;
}

static int wrap(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

/* Row index of the neighbour in direction dy.  Returns -1 when it leaves the
 * lattice (only possible from a solid row, whose stencils are never needed). */
static int nb_row(const ora_params* p, int y, int dy) {
    const int yy = y + dy;
    if (p->bottom == ORA_PERIODIC) return wrap(yy, p->ny);
    return (yy < 0 || yy >= p->ny) ? -1 : yy;
}

/* Equilibrium distribution, Eq 14. */
void ora_feq(double rho, double ux, double uy, double* feq) {
    const double usq = ux * ux + uy * uy;
    for (int i = 0; i < 9; ++i) {
        const double eu = EX[i] * ux + EY[i] * uy;
        feq[i] = rho * W[i] * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * usq);
    }
}

/* Isotropic 9-point Laplacian 6 sum_i w_i (phi(x+e_i) - phi(x)) at (x, y). */
static double lap9(const ora_params* p, const double* phi, int x, int y) {
    const int nx = p->nx;
    double s = 0.0;
    for (int i = 1; i < 9; ++i) {
        const int xx = wrap(x + EX[i], nx), yy = nb_row(p, y, EY[i]);
        s += W[i] * (phi[(size_t)yy * nx + xx] - phi[(size_t)y * nx + x]);
    }
    return 6.0 * s;
}

/* Isotropic gradient 3 sum_i w_i e_i phi(x+e_i) at (x, y). */
static void grad9(const ora_params* p, const double* phi, int x, int y, double* gx, double* gy) {
    const int nx = p->nx;
    double sx = 0.0, sy = 0.0;
    for (int i = 1; i < 9; ++i) {
        const int xx = wrap(x + EX[i], nx), yy = nb_row(p, y, EY[i]);
        const double v = phi[(size_t)yy * nx + xx];
        sx += W[i] * EX[i] * v;
        sy += W[i] * EY[i] * v;
    }
    *gx = 3.0 * sx;
    *gy = 3.0 * sy;
}

/* Stencil probes for the tests (no wall rows: plain periodic wrap). */
void ora_stencils(const ora_params* p, const double* phi, double* lap, double* gx, double* gy) {
    for (int y = 0; y < p->ny; ++y)
        for (int x = 0; x < p->nx; ++x) {
            const size_t c = (size_t)y * p->nx + x;
            if (lap) lap[c] = lap9(p, phi, x, y);
            if (gx && gy) grad9(p, phi, x, y, &gx[c], &gy[c]);
        }
}

/* ------------------------------------------------------------------------ */
/* The pressure-tensor force (Eq 5), the form the paper's Eq 12 replaces       */
/* ------------------------------------------------------------------------ */

/* F = -div(P) + div(P0) with P0 = c_s^2 rho I and the full pressure tensor of
 * Eq 9, P_ab = [p0 - kappa rho lap(rho) - kappa/2 |grad rho|^2] d_ab
 * + kappa d_a rho d_b rho: the three components are formed at every node
 * with the same isotropic stencils, then differentiated once more.  Periodic
 * lattices only (the pressure tensor carries no wall wetting condition). */
static void pressure_tensor_force(const ora_params* p, const double* rho, double* Fx, double* Fy) {
    const int nx = p->nx, ny = p->ny;
    const size_t plane = (size_t)nx * ny;
    double* Pxx = (double*)malloc(3 * plane * sizeof(double));
    double* Pyy = Pxx + plane;
    double* Pxy = Pxx + 2 * plane;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const size_t c = (size_t)y * nx + x;
            double psi, p0, mub, gx, gy;
            eos_eval(p, rho[c], &psi, &p0, &mub);
            grad9(p, rho, x, y, &gx, &gy);
            const double pd = p0 - p->kappa * rho[c] * lap9(p, rho, x, y) - 0.5 * p->kappa * (gx * gx + gy * gy);
            Pxx[c] = pd + p->kappa * gx * gx;
            Pyy[c] = pd + p->kappa * gy * gy;
            Pxy[c] = p->kappa * gx * gy;
        }
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const size_t c = (size_t)y * nx + x;
            double dxx, dyx, dxy, dyy, dxn, dyn, grx, gry;
            grad9(p, Pxx, x, y, &dxx, &dyx);   /* d/dx Pxx (dyx unused) */
            grad9(p, Pxy, x, y, &dxy, &dyy);   /* d/dx Pxy, d/dy Pxy    */
            grad9(p, Pyy, x, y, &dxn, &dyn);   /* d/dy Pyy (dxn unused) */
            grad9(p, rho, x, y, &grx, &gry);
            (void)dyx;
            (void)dxn;
            Fx[c] = -(dxx + dyy) + grx / 3.0;
            Fy[c] = -(dxy + dyn) + gry / 3.0;
        }
    free(Pxx);
}

/* ------------------------------------------------------------------------ */
/* The macroscopic fields of one time level                                  */
/* ------------------------------------------------------------------------ */

/* Computes, for the distributions f of time t (post-streaming), the density
 * (with Eq 28 values in the solid rows), u = sum f e / rho, the chemical
 * potential (Eq 8; wall values in the solid rows) and the force (Eq 12).
 * Solid rows get u = F = 0.  mu_w_bot / mu_w_top hold one value per column
 * and are read only for ORA_CPWALL rows. */
static void macro_fields(const ora_params* p, const double* mu_w_bot, const double* mu_w_top,
                         const double* f, double* rho, double* ux, double* uy, double* mu,
                         double* Fx, double* Fy) {
    const int nx = p->nx, ny = p->ny;
    const size_t plane = (size_t)nx * ny;

    /* 1. moments of the fluid nodes */
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y) {
        if (is_solid_row(p, y)) continue;
        for (int x = 0; x < nx; ++x) {
            const size_t c = (size_t)y * nx + x;
            double r = 0.0, jx = 0.0, jy = 0.0;
            for (int i = 0; i < 9; ++i) {
                r += f[i * plane + c];
                jx += f[i * plane + c] * EX[i];
                jy += f[i * plane + c] * EY[i];
            }
            rho[c] = r;
            ux[c] = jx / r;
            uy[c] = jy / r;
        }
    }

    /* 2. density of the solid rows, Eq 28 (and its mirror at the top) */
    for (int side = 0; side < 2; ++side) {
        const int kind = side == 0 ? p->bottom : p->top;
        if (kind == ORA_PERIODIC) continue;
        const int ys = side == 0 ? 0 : ny - 1;
        const int yf = side == 0 ? 1 : ny - 2;
        for (int x = 0; x < nx; ++x) {
            const double r0 = rho[(size_t)yf * nx + x];
            const double rl = rho[(size_t)yf * nx + wrap(x - 1, nx)];
            const double rr = rho[(size_t)yf * nx + wrap(x + 1, nx)];
            rho[(size_t)ys * nx + x] = 2.0 / 3.0 * r0 + 1.0 / 6.0 * rl + 1.0 / 6.0 * rr;
            ux[(size_t)ys * nx + x] = 0.0;
            uy[(size_t)ys * nx + x] = 0.0;
        }
    }

    /* 3. chemical potential, Eq 8, at the fluid nodes */
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y) {
        if (is_solid_row(p, y)) continue;
        for (int x = 0; x < nx; ++x) {
            const size_t c = (size_t)y * nx + x;
            double psi, p0, mub;
            eos_eval(p, rho[c], &psi, &p0, &mub);
            mu[c] = mub - p->kappa * lap9(p, rho, x, y);
        }
    }
    /* wall chemical potential: the surface value (Sec. IV) or a copy of the
       neighbouring fluid node (Sec. V, top side) */
    for (int side = 0; side < 2; ++side) {
        const int kind = side == 0 ? p->bottom : p->top;
        if (kind == ORA_PERIODIC) continue;
        const int ys = side == 0 ? 0 : ny - 1;
        const int yf = side == 0 ? 1 : ny - 2;
        const double* mw = side == 0 ? mu_w_bot : mu_w_top;
        for (int x = 0; x < nx; ++x)
            mu[(size_t)ys * nx + x] = kind == ORA_CPWALL ? mw[x] : mu[(size_t)yf * nx + x];
    }

    if ((p->scheme & 15) == ORA_FORCE_PTENSOR) {
        pressure_tensor_force(p, rho, Fx, Fy);
        return;
    }

    /* 4. nonideal force, Eq 12 with div(P0) = c_s^2 grad(rho), c_s^2 = 1/3 */
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            const size_t c = (size_t)y * nx + x;
            if (is_solid_row(p, y)) {
                Fx[c] = 0.0;
                Fy[c] = 0.0;
                continue;
            }
            double gmx, gmy, grx, gry;
            grad9(p, mu, x, y, &gmx, &gmy);
            grad9(p, rho, x, y, &grx, &gry);
            Fx[c] = -rho[c] * gmx + grx / 3.0;
            Fy[c] = -rho[c] * gmy + gry / 3.0;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Collision of one node                                                      */
/* ------------------------------------------------------------------------ */

/* MRT moments of Lallemand and Luo: rho, e, epsilon, j_x, q_x, j_y, q_y,
 * p_xx, p_xy, as rows over the directions 0..8.  The rows are orthogonal, so
 * the inverse transform is M^T diag(1 / |row|^2). */
static const double MRT_M[9][9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-4, -1, -1, -1, -1, 2, 2, 2, 2},
    {4, -2, -2, -2, -2, 1, 1, 1, 1},
    {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, -2, 0, 2, 0, 1, -1, -1, 1},
    {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},
    {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1}};

void ora_mrt_matrix(double* out) { memcpy(out, MRT_M, sizeof MRT_M); }

/* Post-collision f* of one fluid node with density r, velocity (ux, uy) and
 * force (Fx, Fy).  The force enters through the equilibrium velocity (forcing
 * paragraph after Eq 14), shifted by tau F / rho for BGK.  With several
 * relaxation times each relaxing part is shifted by its own relaxation time,
 * F / (rho s): the even part of TRT by tau F / rho and its odd part by
 * tau- F / rho, each MRT moment k by F / (rho s_k).  Every part then gains from
 * the force what it gains under BGK (in particular the momentum gains exactly
 * F), and equal relaxation times give BGK. */
static void collide_node(const ora_params* p, const double* f, double r, double ux, double uy, double Fx,
                         double Fy, double* fs) {
    const double tau = p->tau;
    const int coll = p->scheme & 0xf0;
    if (coll == ORA_COLLIDE_TRT) {
        const double tm = 0.5 + p->trt_lambda / (tau - 0.5);   /* tau- */
        double fe[9], fo[9];
        ora_feq(r, ux + tau * Fx / r, uy + tau * Fy / r, fe);   /* even part's equilibrium */
        ora_feq(r, ux + tm * Fx / r, uy + tm * Fy / r, fo);     /* odd part's equilibrium  */
        for (int i = 0; i < 9; ++i) {
            const int o = OPP[i];
            const double sp = 0.5 * (f[i] + f[o]) - 0.5 * (fe[i] + fe[o]);
            const double sm = 0.5 * (f[i] - f[o]) - 0.5 * (fo[i] - fo[o]);
            fs[i] = f[i] - sp / tau - sm / tm;
        }
        return;
    }
    if (coll == ORA_COLLIDE_MRT) {
        const double sn = 1.0 / tau;
        const double S[9] = {sn, p->s_e, p->s_eps, sn, p->s_q, sn, p->s_q, sn, sn};
        double dm[9];
        for (int k = 0; k < 9; ++k) {
            double feq[9];
            ora_feq(r, ux + Fx / (r * S[k]), uy + Fy / (r * S[k]), feq);
            double norm = 0.0, m = 0.0, meq = 0.0;
            for (int i = 0; i < 9; ++i) {
                norm += MRT_M[k][i] * MRT_M[k][i];
                m += MRT_M[k][i] * f[i];
                meq += MRT_M[k][i] * feq[i];
            }
            dm[k] = S[k] * (m - meq) / norm;
        }
        for (int i = 0; i < 9; ++i) {
            double d = 0.0;
            for (int k = 0; k < 9; ++k) d += MRT_M[k][i] * dm[k];
            fs[i] = f[i] - d;
        }
        return;
    }
    double feq[9];
    ora_feq(r, ux + tau * Fx / r, uy + tau * Fy / r, feq);
    for (int i = 0; i < 9; ++i) fs[i] = f[i] - (f[i] - feq[i]) / tau;  /* BGK, Eq 13 */
}

/* ------------------------------------------------------------------------ */
/* Public oracle entry points                                                */
/* ------------------------------------------------------------------------ */

/* f = f_eq(rho0, u0) at every fluid node (u0 = 0 when ux0/uy0 are NULL);
 * solid rows are zero.  f is [9][ny][nx]. */
void ora_init(const ora_params* p, const double* rho0, const double* ux0, const double* uy0,
              double* f) {
    const int nx = p->nx, ny = p->ny;
    const size_t plane = (size_t)nx * ny;
    memset(f, 0, 9 * plane * sizeof(double));
    for (int y = 0; y < ny; ++y) {
        if (is_solid_row(p, y)) continue;
        for (int x = 0; x < nx; ++x) {
            const size_t c = (size_t)y * nx + x;
            double feq[9];
            ora_feq(rho0[c], ux0 ? ux0[c] : 0.0, uy0 ? uy0[c] : 0.0, feq);
            for (int i = 0; i < 9; ++i) f[i * plane + c] = feq[i];
        }
    }
}

/* One time step f(t) -> fnew(t+1) (Eq 13).  work must hold 7 * nx * ny
 * doubles; on return it holds rho, ux, uy, mu, Fx, Fy of time t (planes 0..5). */
void ora_step(const ora_params* p, const double* mu_w_bot, const double* mu_w_top,
              const double* f, double* fnew, double* work) {
    const int nx = p->nx, ny = p->ny;
    const size_t plane = (size_t)nx * ny;
    double *rho = work, *ux = work + plane, *uy = work + 2 * plane, *mu = work + 3 * plane;
    double *Fx = work + 4 * plane, *Fy = work + 5 * plane;
    macro_fields(p, mu_w_bot, mu_w_top, f, rho, ux, uy, mu, Fx, Fy);

    memset(fnew, 0, 9 * plane * sizeof(double));
    /* 5-6. collision with the shifted equilibrium velocity, then streaming */
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y) {
        if (is_solid_row(p, y)) continue;
        for (int x = 0; x < nx; ++x) {
            const size_t c = (size_t)y * nx + x;
            double fin[9], fout[9];
            for (int i = 0; i < 9; ++i) fin[i] = f[i * plane + c];
            collide_node(p, fin, rho[c], ux[c], uy[c], Fx[c], Fy[c], fout);
            for (int i = 0; i < 9; ++i) {
                const double fstar = fout[i];
                const int xt = wrap(x + EX[i], nx);
                const int yt = nb_row(p, y, EY[i]);
                if (yt < 0 || is_solid_row(p, yt)) {
                    /* halfway bounce-back: returns to the same node reversed */
                    fnew[OPP[i] * plane + c] = fstar;
                } else {
                    /* each target slot has exactly one source, so no race */
                    fnew[i * plane + (size_t)yt * nx + xt] = fstar;
                }
            }
        }
    }
}

/* nsteps steps in place on f, using fbuf (9 * nx * ny) and work (7 * nx * ny). */
void ora_run(const ora_params* p, const double* mu_w_bot, const double* mu_w_top, double* f,
             double* fbuf, double* work, int64_t nsteps) {
    const size_t n = (size_t)9 * p->nx * p->ny;
    for (int64_t s = 0; s < nsteps; ++s) {
        ora_step(p, mu_w_bot, mu_w_top, f, fbuf, work);
        memcpy(f, fbuf, n * sizeof(double));
    }
}

/* Output fields of the state f: rho (Eq 28 values in solid rows), the
 * physical velocity v = u + F / (2 rho), the chemical potential and the force.
 * work must hold 7 * nx * ny doubles.  Any output pointer may be NULL. */
void ora_fields(const ora_params* p, const double* mu_w_bot, const double* mu_w_top,
                const double* f, double* rho, double* vx, double* vy, double* mu, double* Fx,
                double* Fy, double* work) {
    const int nx = p->nx, ny = p->ny;
    const size_t plane = (size_t)nx * ny;
    double *r = work, *ux = work + plane, *uy = work + 2 * plane, *m = work + 3 * plane;
    double *fx = work + 4 * plane, *fy = work + 5 * plane;
    macro_fields(p, mu_w_bot, mu_w_top, f, r, ux, uy, m, fx, fy);
    for (size_t c = 0; c < plane; ++c) {
        const int y = (int)(c / nx);
        const int solid = is_solid_row(p, y);
        if (rho) rho[c] = r[c];
        if (vx) vx[c] = solid ? 0.0 : ux[c] + fx[c] / (2.0 * r[c]);
        if (vy) vy[c] = solid ? 0.0 : uy[c] + fy[c] / (2.0 * r[c]);
        if (mu) mu[c] = m[c];
        if (Fx) Fx[c] = fx[c];
        if (Fy) Fy[c] = fy[c];
    }
}

/* Total mass sum_i f_i over the fluid nodes, serial fixed order. */
double ora_mass(const ora_params* p, const double* f) {
    const size_t plane = (size_t)p->nx * p->ny;
    double m = 0.0;
    for (int y = 0; y < p->ny; ++y) {
        if (is_solid_row(p, y)) continue;
        for (int x = 0; x < p->nx; ++x)
            for (int i = 0; i < 9; ++i) m += f[i * plane + (size_t)y * p->nx + x];
    }
    return m;
}

int ora_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void ora_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
