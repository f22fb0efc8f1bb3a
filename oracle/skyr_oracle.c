/*
 * skyr_oracle.c -- plain, slow, FP64 CPU reference for the arrested Newton
 * flow of the 3D Skyrme model in the sigma-model (unit 4-vector) form.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header or table with the HIP path.
 *
 * Every routine follows a passage of arXiv:2604.25876 (cuSkyrmion):
 *   - energy density:      Sec. 2.1, eq. (SkyrmeEnergy_phi), taken at one half
 *                          of the printed normalisation, discretised with the
 *                          two fourth-order stencils of Sec. 3:
 *                          e = -1/2 phi.Lap_h phi + 1/4 (S^2 - sum_ij G_ij^2) + m^2 (1 - phi^0)
 *                          (for unit fields -phi.Lap phi = |d phi|^2 in the continuum)
 *   - baryon density:      Sec. 2.1, eq. (B0_components)
 *   - Newton flow:         Sec. 3, eq. (Newton_flow) with the tangent projection
 *   - arrest / stop rule:  Sec. 3, the paragraphs after eq. (Sigma model EL equations)
 *   - renormalisation:     Sec. 3, explicit projection phi <- phi/|phi|
 *   - lattice + stencils:  Sec. 3, fourth-order first and second differences;
 *                          the energy is a function on the lattice values
 *   - rational maps:       Sec. 4.1 and Table (RMA)
 *   - product ansatz:      Sec. 4.2, eq. (Product ansatz)
 *   - isorotation D(A):    Sec. 5.3, the SU(2) -> SO(3) homomorphism
 *
 * Conventions (readings of the paper, listed in the design notes):
 *   - field layout phi[A][x][y][z], A = 0..3, z fastest, n[0] x n[1] x n[2];
 *   - coordinates x_i = (i - (n-1)/2) h;
 *   - two frozen vacuum layers per face; the interior I = {2..n-3}^3 carries
 *     the energy, the charge and the update;
 *   - a_i = D_i phi (first-difference stencil), G_ij = a_i.a_j, S = tr G,
 *     Lap_h = sum_i (five-point second difference along i);
 *   - the discrete gradient is the exact derivative of the discrete energy
 *     E_h = h^3 sum_{x in I} e(x):
 *        g = -1/2 (Lap_h phi + Lap_h(1_I phi)) - sum_i D_i Q_i - m^2 e_0
 *     in density units (g = h^-3 dE_h/dphi), with the quartic flux
 *     Q_i = S a_i - sum_j G_ij a_j = d e4 / d a_i and Q = 0 outside I;
 *   - baryon density b = -(1/2 pi^2) det[phi, a_1, a_2, a_3] so that the
 *     hedgehog with f(0) = pi has B = +1;
 *   - arrest when E(phi_n) > E(phi_{n-1}) (strict), v_n <- 0, field kept.
 *
 * Sums are deterministic: each x-plane is summed serially in (y, z) order and
 * the plane sums are added serially in x order, whatever the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_API __attribute__((visibility("default")))

/* ------------------------------------------------------------------------ */
/* indexing                                                                 */
/* ------------------------------------------------------------------------ */

static size_t n_sites(const int n[3]) { return (size_t)n[0] * n[1] * n[2]; }

static size_t site(const int n[3], int x, int y, int z)
{
    return ((size_t)x * n[1] + y) * n[2] + z;
}

static int interior(const int n[3], int x, int y, int z)
{
    return x >= 2 && x <= n[0] - 3 && y >= 2 && y <= n[1] - 3 && z >= 2 && z <= n[2] - 3;
}

/* component A of a [4][n0][n1][n2] array */
#define FLD(arr, A, s) ((arr)[(size_t)(A) * N3 + (s)])

/* ------------------------------------------------------------------------ */
/* Sec. 3: fourth-order first derivative                                    */
/*   d_x f_i = ( -1/12 f_{i+2} + 2/3 f_{i+1} - 2/3 f_{i-1} + 1/12 f_{i-2} ) / h */
/* ------------------------------------------------------------------------ */

static double d1(const double *f, const int n[3], int axis, int x, int y, int z, double h)
{
    int dx = axis == 0, dy = axis == 1, dz = axis == 2;
    double fp1 = f[site(n, x + dx, y + dy, z + dz)];
    double fm1 = f[site(n, x - dx, y - dy, z - dz)];
    double fp2 = f[site(n, x + 2 * dx, y + 2 * dy, z + 2 * dz)];
    double fm2 = f[site(n, x - 2 * dx, y - 2 * dy, z - 2 * dz)];
    /* the same stencil written as differences of mirrored neighbours */
    return (2.0 / 3.0 * (fp1 - fm1) - 1.0 / 12.0 * (fp2 - fm2)) / h;
}

/* Sec. 3: fourth-order (five-point) second derivative. */
static double d2(const double *f, const int n[3], int axis, int x, int y, int z, double h)
{
    int dx = axis == 0, dy = axis == 1, dz = axis == 2;
    double f0 = f[site(n, x, y, z)];
    double fp1 = f[site(n, x + dx, y + dy, z + dz)];
    double fm1 = f[site(n, x - dx, y - dy, z - dz)];
    double fp2 = f[site(n, x + 2 * dx, y + 2 * dy, z + 2 * dz)];
    double fm2 = f[site(n, x - 2 * dx, y - 2 * dy, z - 2 * dz)];
    return (4.0 / 3.0 * (fp1 + fm1) - 1.0 / 12.0 * (fp2 + fm2) - 5.0 / 2.0 * f0) / (h * h);
}

/* a[i][A] = D_i phi^A at one site (any site at least two layers from the faces) */
static void derivs_at(const double *phi, const int n[3], double h, int x, int y, int z, double a[3][4])
{
    const size_t N3 = n_sites(n);
    for (int i = 0; i < 3; i++)
        for (int A = 0; A < 4; A++)
            a[i][A] = d1(phi + (size_t)A * N3, n, i, x, y, z, h);
}

/* D_i applied to component A of every interior site; zero outside I.
 * Output layout a[i][A][site], i.e. 12 arrays of n0*n1*n2 doubles. */
ORA_API void ora_first_derivatives(const int n[3], double h, const double *phi, double *a)
{
    const size_t N3 = n_sites(n);
    memset(a, 0, 12 * N3 * sizeof(double));
#pragma omp parallel for schedule(static)
    for (int x = 2; x <= n[0] - 3; x++)
        for (int y = 2; y <= n[1] - 3; y++)
            for (int z = 2; z <= n[2] - 3; z++) {
                size_t s = site(n, x, y, z);
                for (int i = 0; i < 3; i++)
                    for (int A = 0; A < 4; A++)
                        a[((size_t)i * 4 + A) * N3 + s] = d1(phi + (size_t)A * N3, n, i, x, y, z, h);
            }
}

/* Lap_h phi^A (sum of the three five-point second differences) on the
 * interior, zero elsewhere; layout [4][n0][n1][n2]. */
static void laplacian_at(const double *phi, const int n[3], double h, int x, int y, int z, double lap[4]);

ORA_API void ora_laplacian(const int n[3], double h, const double *phi, double *lap)
{
    const size_t N3 = n_sites(n);
    memset(lap, 0, 4 * N3 * sizeof(double));
#pragma omp parallel for schedule(static)
    for (int x = 2; x <= n[0] - 3; x++)
        for (int y = 2; y <= n[1] - 3; y++)
            for (int z = 2; z <= n[2] - 3; z++) {
                double l[4];
                laplacian_at(phi, n, h, x, y, z, l);
                for (int A = 0; A < 4; A++) FLD(lap, A, site(n, x, y, z)) = l[A];
            }
}

/* ------------------------------------------------------------------------ */
/* Sec. 2.1: energy density (one half of the printed normalisation)         */
/* ------------------------------------------------------------------------ */

static double dot4(const double *u, const double *v)
{
    return u[0] * v[0] + u[1] * v[1] + u[2] * v[2] + u[3] * v[3];
}

static double det4(const double c0[4], const double c1[4], const double c2[4], const double c3[4]);

/* Sextic (BPS-Skyrme) term at one interior site (Sec. 7.7: c6 4 pi^4 (B0)^2 in the
 * printed normalisation, halved here, with B0 = b = -(1/2 pi^2) det[phi, a_1, a_2, a_3]):
 *   e6 = c6 det^2 / 2.
 * det is linear in each column, so its derivative with respect to column k is the
 * determinant with that column replaced by the unit vector e_A.  Returns det and
 * fills C[k][A] = d det / d(column k)_A, k = 0 (phi), 1..3 (a_1..a_3). */
static double det_and_cofactors(const double p[4], double a[3][4], double C[4][4])
{
    static const double E[4][4] = {{1, 0, 0, 0}, {0, 1, 0, 0}, {0, 0, 1, 0}, {0, 0, 0, 1}};
    for (int A = 0; A < 4; A++) {
        C[0][A] = det4(E[A], a[0], a[1], a[2]);
        C[1][A] = det4(p, E[A], a[1], a[2]);
        C[2][A] = det4(p, a[0], E[A], a[2]);
        C[3][A] = det4(p, a[0], a[1], E[A]);
    }
    return det4(p, a[0], a[1], a[2]);
}

/* Lap_h phi^A at one site: sum over the three axes of the five-point second difference */
static void laplacian_at(const double *phi, const int n[3], double h, int x, int y, int z, double lap[4])
{
    const size_t N3 = n_sites(n);
    for (int A = 0; A < 4; A++) {
        double t = 0.0;
        for (int i = 0; i < 3; i++) t += d2(phi + (size_t)A * N3, n, i, x, y, z, h);
        lap[A] = t;
    }
}

/* Potential density of phi0 (Sec. 7.7, the four potentials of the program, in this
 * energy's normalisation, i.e. halved):
 *   V = m_x^2 (1 - phi0) + m_y^2 (1 - phi0^2)/2 + m_z^2 (1 - phi0)^2/2 + m_w^2 (1 - phi0)^4/4
 * mass = {m_x, m_y, m_z, m_w, c6} (the model constants); m_x is the pion mass m of Sec. 2.1. */
static double potential(const double *mass, double p0)
{
    double u = 1.0 - p0;
    return mass[0] * mass[0] * u + 0.5 * mass[1] * mass[1] * (1.0 - p0 * p0) + 0.5 * mass[2] * mass[2] * u * u +
           0.25 * mass[3] * mass[3] * u * u * u * u;
}

/* dV/dphi0 */
static double potential_slope(const double *mass, double p0)
{
    double u = 1.0 - p0;
    return -mass[0] * mass[0] - mass[1] * mass[1] * p0 - mass[2] * mass[2] * u - mass[3] * mass[3] * u * u * u;
}

/* e2 = -1/2 phi.Lap_h phi;  G_ij = a_i . a_j, S = tr G, e4 = (S^2 - sum_ij G_ij^2)/4;
 * e0 = V(phi0) */
static void density_parts(const double p[4], const double lap[4], double a[3][4], const double *mass, double *e2,
                          double *e4, double *e0)
{
    double G[3][3];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            G[i][j] = dot4(a[i], a[j]);
    double S = G[0][0] + G[1][1] + G[2][2];
    double GG = 0.0;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            GG += G[i][j] * G[i][j];
    *e2 = -0.5 * dot4(p, lap);
    *e4 = 0.25 * (S * S - GG);
    *e0 = potential(mass, p[0]);
}

/* E2, E4, E0 = h^3 sum over I of the three parts (deterministic order). */
/* E2, E4, E0, E6 = h^3 sum over I of the four parts (deterministic order).
 * model = {m, m_y, m_z, m_w, c6}. */
ORA_API void ora_energy_parts(const int n[3], double h, const double *model, const double *phi, double out[4])
{
    const size_t N3 = n_sites(n);
    const double c6 = model[4];
    double *plane = calloc((size_t)n[0] * 4, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int x = 2; x <= n[0] - 3; x++) {
        double s2 = 0.0, s4 = 0.0, s0 = 0.0, s6 = 0.0;
        for (int y = 2; y <= n[1] - 3; y++)
            for (int z = 2; z <= n[2] - 3; z++) {
                double a[3][4], lap[4], p[4], e2, e4, e0;
                size_t s = site(n, x, y, z);
                for (int A = 0; A < 4; A++) p[A] = FLD(phi, A, s);
                derivs_at(phi, n, h, x, y, z, a);
                laplacian_at(phi, n, h, x, y, z, lap);
                density_parts(p, lap, a, model, &e2, &e4, &e0);
                s2 += e2;
                s4 += e4;
                s0 += e0;
                if (c6 != 0.0) {
                    double d = det4(p, a[0], a[1], a[2]);
                    s6 += 0.5 * c6 * d * d;
                }
            }
        plane[4 * x + 0] = s2;
        plane[4 * x + 1] = s4;
        plane[4 * x + 2] = s0;
        plane[4 * x + 3] = s6;
    }
    double t2 = 0.0, t4 = 0.0, t0 = 0.0, t6 = 0.0;
    for (int x = 0; x < n[0]; x++) {
        t2 += plane[4 * x + 0];
        t4 += plane[4 * x + 1];
        t0 += plane[4 * x + 2];
        t6 += plane[4 * x + 3];
    }
    free(plane);
    double h3 = h * h * h;
    out[0] = h3 * t2;
    out[1] = h3 * t4;
    out[2] = h3 * t0;
    out[3] = h3 * t6;
}

ORA_API double ora_energy(const int n[3], double h, const double *model, const double *phi)
{
    double p[4];
    ora_energy_parts(n, h, model, phi, p);
    return p[0] + p[1] + p[2] + p[3];
}

/* ------------------------------------------------------------------------ */
/* exact discrete gradient (derivative of E_h with respect to lattice values) */
/* ------------------------------------------------------------------------ */

/* quartic flux Q_i^A = de4/da_i^A = S a_i^A - sum_j G_ij a_j^A */
static void flux_from_derivs(double a[3][4], double P[3][4])
{
    double G[3][3];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            G[i][j] = dot4(a[i], a[j]);
    double S = G[0][0] + G[1][1] + G[2][2];
    for (int i = 0; i < 3; i++)
        for (int A = 0; A < 4; A++) {
            double t = S * a[i][A];
            for (int j = 0; j < 3; j++)
                t -= G[i][j] * a[j][A];
            P[i][A] = t;
        }
}

/* Quartic flux at every site: Q[i][A][site], zero outside I. */
ORA_API void ora_flux(const int n[3], double h, const double *phi, double *P)
{
    const size_t N3 = n_sites(n);
    memset(P, 0, 12 * N3 * sizeof(double));
#pragma omp parallel for schedule(static)
    for (int x = 2; x <= n[0] - 3; x++)
        for (int y = 2; y <= n[1] - 3; y++)
            for (int z = 2; z <= n[2] - 3; z++) {
                double a[3][4], Pl[3][4];
                derivs_at(phi, n, h, x, y, z, a);
                flux_from_derivs(a, Pl);
                size_t s = site(n, x, y, z);
                for (int i = 0; i < 3; i++)
                    for (int A = 0; A < 4; A++)
                        P[((size_t)i * 4 + A) * N3 + s] = Pl[i][A];
            }
}

/* g(y) at interior y, 0 on the frozen layers; g is h^-3 times the derivative
 * of E_h with respect to phi(y):
 *   E2 part:  d/dphi(y) of -1/2 sum_{x in I} phi(x).Lap phi(x)
 *             = -1/2 (1_I(y) Lap phi(y) + Lap(1_I phi)(y))       (Lap symmetric)
 *   E4 part:  sum over x in I and axis i of Q_i(x) da_i(x)/dphi(y) = -D_i Q_i(y)
 *             (D antisymmetric, Q = 0 outside I)
 *   E0 part:  dV/dphi0 e_0. */
ORA_API void ora_gradient(const int n[3], double h, const double *mass, const double *phi, double *g)
{
    const size_t N3 = n_sites(n);
    const double c6 = mass[4];
    double *P = malloc(12 * N3 * sizeof(double));
    double *phiI = malloc(4 * N3 * sizeof(double));
    ora_flux(n, h, phi, P);
    /* sextic part: flux c6 det C_i added to the quartic flux (zero outside I), local
     * term c6 det C_0 at the site itself */
    double *L6 = calloc(4 * N3, sizeof(double));
    if (c6 != 0.0) {
#pragma omp parallel for schedule(static)
        for (int x = 2; x <= n[0] - 3; x++)
            for (int y = 2; y <= n[1] - 3; y++)
                for (int z = 2; z <= n[2] - 3; z++) {
                    size_t s = site(n, x, y, z);
                    double a[3][4], p[4], C[4][4];
                    derivs_at(phi, n, h, x, y, z, a);
                    for (int A = 0; A < 4; A++) p[A] = FLD(phi, A, s);
                    double d = det_and_cofactors(p, a, C);
                    for (int A = 0; A < 4; A++) {
                        for (int i = 0; i < 3; i++) P[((size_t)i * 4 + A) * N3 + s] += c6 * d * C[i + 1][A];
                        FLD(L6, A, s) = c6 * d * C[0][A];
                    }
                }
    }
    /* 1_I phi: the field with every site outside the interior set to zero */
    for (int A = 0; A < 4; A++)
        for (int x = 0; x < n[0]; x++)
            for (int y = 0; y < n[1]; y++)
                for (int z = 0; z < n[2]; z++) {
                    size_t s = site(n, x, y, z);
                    FLD(phiI, A, s) = interior(n, x, y, z) ? FLD(phi, A, s) : 0.0;
                }
    memset(g, 0, 4 * N3 * sizeof(double));
#pragma omp parallel for schedule(static)
    for (int x = 2; x <= n[0] - 3; x++)
        for (int y = 2; y <= n[1] - 3; y++)
            for (int z = 2; z <= n[2] - 3; z++) {
                size_t s = site(n, x, y, z);
                double lap[4], lapI[4];
                laplacian_at(phi, n, h, x, y, z, lap);
                laplacian_at(phiI, n, h, x, y, z, lapI);
                for (int A = 0; A < 4; A++) {
                    double div = 0.0;
                    for (int i = 0; i < 3; i++)
                        div += d1(P + ((size_t)i * 4 + A) * N3, n, i, x, y, z, h);
                    FLD(g, A, s) = -0.5 * (lap[A] + lapI[A]) - div + FLD(L6, A, s) +
                                   (A == 0 ? potential_slope(mass, FLD(phi, 0, s)) : 0.0);
                }
            }
    free(P);
    free(phiI);
    free(L6);
}

/* Tangent projection (Sec. 3, eq. Newton_flow): gT = g - (g.phi) phi on I.
 * The Newton-flow force is F = -gT.  Returns max over I of |gT|. */
ORA_API double ora_project(const int n[3], const double *phi, const double *g, double *gT)
{
    const size_t N3 = n_sites(n);
    double *pm = calloc((size_t)n[0], sizeof(double));
    memset(gT, 0, 4 * N3 * sizeof(double));
#pragma omp parallel for schedule(static)
    for (int x = 2; x <= n[0] - 3; x++) {
        double mx = 0.0;
        for (int y = 2; y <= n[1] - 3; y++)
            for (int z = 2; z <= n[2] - 3; z++) {
                size_t s = site(n, x, y, z);
                double gp = 0.0;
                for (int A = 0; A < 4; A++)
                    gp += FLD(g, A, s) * FLD(phi, A, s);
                double nrm2 = 0.0;
                for (int A = 0; A < 4; A++) {
                    double t = FLD(g, A, s) - gp * FLD(phi, A, s);
                    FLD(gT, A, s) = t;
                    nrm2 += t * t;
                }
                double nr = sqrt(nrm2);
                if (nr > mx || isnan(nr)) mx = nr;
            }
        pm[x] = mx;
    }
    double r = 0.0;
    for (int x = 0; x < n[0]; x++)
        if (pm[x] > r || isnan(pm[x])) r = pm[x];
    free(pm);
    return r;
}

/* The same gradient at one interior site, computed locally from the
 * definition (quartic flux at the twelve stencil neighbours, Laplacians of
 * phi and of 1_I phi).  Used to check single outputs of large lattices. */
ORA_API void ora_gradient_at(const int n[3], double h, const double *mass, const double *phi, int x, int y, int z,
                             double g[4])
{
    const size_t N3 = n_sites(n);
    static const int off[4] = {-2, -1, 1, 2};
    /* D_i f(y) = sum_k c1[k] f(y + off[k] e_i) / h;  d2: c2[k] / h^2 off the centre */
    static const double c1[4] = {1.0 / 12.0, -2.0 / 3.0, 2.0 / 3.0, -1.0 / 12.0};
    static const double c2[4] = {-1.0 / 12.0, 4.0 / 3.0, 4.0 / 3.0, -1.0 / 12.0};
    double div[4] = {0, 0, 0, 0}, lap[4], lapI[4];
    laplacian_at(phi, n, h, x, y, z, lap);
    size_t s0 = site(n, x, y, z);
    for (int A = 0; A < 4; A++) lapI[A] = 3.0 * (-5.0 / 2.0) * FLD(phi, A, s0) / (h * h);
    for (int i = 0; i < 3; i++)
        for (int k = 0; k < 4; k++) {
            int xx = x + (i == 0) * off[k], yy = y + (i == 1) * off[k], zz = z + (i == 2) * off[k];
            if (!interior(n, xx, yy, zz)) continue; /* Q = 0 and 1_I phi = 0 outside I */
            double a[3][4], P[3][4];
            derivs_at(phi, n, h, xx, yy, zz, a);
            flux_from_derivs(a, P);
            size_t s = site(n, xx, yy, zz);
            if (mass[4] != 0.0) {
                double pp[4], C[4][4];
                for (int A = 0; A < 4; A++) pp[A] = FLD(phi, A, s);
                double d = det_and_cofactors(pp, a, C);
                for (int ii = 0; ii < 3; ii++)
                    for (int A = 0; A < 4; A++) P[ii][A] += mass[4] * d * C[ii + 1][A];
            }
            for (int A = 0; A < 4; A++) {
                div[A] += c1[k] * P[i][A] / h;
                lapI[A] += c2[k] * FLD(phi, A, s) / (h * h);
            }
        }
    double L6[4] = {0, 0, 0, 0};
    if (mass[4] != 0.0) {
        double a[3][4], pp[4], C[4][4];
        derivs_at(phi, n, h, x, y, z, a);
        for (int A = 0; A < 4; A++) pp[A] = FLD(phi, A, s0);
        double d = det_and_cofactors(pp, a, C);
        for (int A = 0; A < 4; A++) L6[A] = mass[4] * d * C[0][A];
    }
    for (int A = 0; A < 4; A++)
        g[A] = -0.5 * (lap[A] + lapI[A]) - div[A] + L6[A] + (A == 0 ? potential_slope(mass, FLD(phi, 0, s0)) : 0.0);
}

/* ------------------------------------------------------------------------ */
/* Sec. 2.1: baryon density and number                                      */
/* ------------------------------------------------------------------------ */

static double det4(const double c0[4], const double c1[4], const double c2[4], const double c3[4])
{
    /* Laplace expansion along the first column: det[c0 c1 c2 c3] */
    double m[4][4];
    for (int r = 0; r < 4; r++) {
        m[r][0] = c0[r];
        m[r][1] = c1[r];
        m[r][2] = c2[r];
        m[r][3] = c3[r];
    }
    double det = 0.0;
    for (int r = 0; r < 4; r++) {
        double sub[3][3];
        int rr = 0;
        for (int k = 0; k < 4; k++) {
            if (k == r) continue;
            for (int c = 0; c < 3; c++) sub[rr][c] = m[k][c + 1];
            rr++;
        }
        double d3 = sub[0][0] * (sub[1][1] * sub[2][2] - sub[1][2] * sub[2][1]) -
                    sub[0][1] * (sub[1][0] * sub[2][2] - sub[1][2] * sub[2][0]) +
                    sub[0][2] * (sub[1][0] * sub[2][1] - sub[1][1] * sub[2][0]);
        det += ((r % 2) ? -1.0 : 1.0) * m[r][0] * d3;
    }
    return det;
}

/* b = -(1/(2 pi^2)) det[phi, a_1, a_2, a_3]: the epsilon^{ijk} epsilon_{ABCD}
 * contraction equals 3! times the determinant; the overall sign is chosen so
 * that the hedgehog with f(0) = pi carries B = +1. */
static double baryon_density_at(const double *phi, const int n[3], double h, int x, int y, int z)
{
    const size_t N3 = n_sites(n);
    double a[3][4], p[4];
    derivs_at(phi, n, h, x, y, z, a);
    size_t s = site(n, x, y, z);
    for (int A = 0; A < 4; A++) p[A] = FLD(phi, A, s);
    return -det4(p, a[0], a[1], a[2]) / (2.0 * M_PI * M_PI);
}

ORA_API double ora_baryon(const int n[3], double h, const double *phi)
{
    double *plane = calloc((size_t)n[0], sizeof(double));
#pragma omp parallel for schedule(static)
    for (int x = 2; x <= n[0] - 3; x++) {
        double s = 0.0;
        for (int y = 2; y <= n[1] - 3; y++)
            for (int z = 2; z <= n[2] - 3; z++)
                s += baryon_density_at(phi, n, h, x, y, z);
        plane[x] = s;
    }
    double t = 0.0;
    for (int x = 0; x < n[0]; x++) t += plane[x];
    free(plane);
    return h * h * h * t;
}

/* Observables: E2, E4, E0, E6, E, B, virial V = E2 - E4 + 3 E0 - 3 E6 (Sec. 5.6;
 * the Derrick scaling argument: under x -> lambda x the parts scale as
 * lambda^-1, lambda, lambda^-3, lambda^3), and the largest tangential gradient
 * norm.  out = {E, E2, E4, E0, B, virial, max_force, E6}. */
ORA_API void ora_observables(const int n[3], double h, const double *mass, const double *phi, double out[8])
{
    const size_t N3 = n_sites(n);
    double p[4];
    ora_energy_parts(n, h, mass, phi, p);
    double *g = malloc(4 * N3 * sizeof(double));
    double *gT = malloc(4 * N3 * sizeof(double));
    ora_gradient(n, h, mass, phi, g);
    double r = ora_project(n, phi, g, gT);
    free(g);
    free(gT);
    out[0] = p[0] + p[1] + p[2] + p[3];
    out[1] = p[0];
    out[2] = p[1];
    out[3] = p[2];
    out[4] = ora_baryon(n, h, phi);
    out[5] = p[0] - p[1] + 3.0 * p[2] - 3.0 * p[3];
    out[6] = r;
    out[7] = p[3];
}

/* ------------------------------------------------------------------------ */
/* Sec. 3: arrested Newton flow                                             */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t steps;     /* accepted updates so far (n)                           */
    int64_t arrests;   /* number of velocity resets                            */
    double E_prev;     /* E(phi_{n-1}); +inf before the first update           */
    double E;          /* E(phi_n) at the last evaluated step                  */
    double max_force;  /* max over I of |F(phi_n)| at the last evaluated step  */
    int32_t converged; /* 1 once max_force < tol                               */
    int32_t nonfinite; /* 1 if E or max_force stopped being finite             */
} ora_anf_state;

/* One kick-drift (symplectic Euler) step at a site with renormalisation:
 * v' = v + dt F,  phi' = (phi + dt v') / |phi + dt v'|. */
static void kick_drift(double *p, double *v, const double F[4], double dt)
{
    double q[4], nrm2 = 0.0;
    for (int A = 0; A < 4; A++) {
        v[A] = v[A] + dt * F[A];
        q[A] = p[A] + dt * v[A];
        nrm2 += q[A] * q[A];
    }
    double nr = sqrt(nrm2);
    for (int A = 0; A < 4; A++) p[A] = q[A] / nr;
}

/* Single-site form of one update for sampled checks: given phi, v and the
 * (unprojected) gradient g at a site, returns phi' and v'. */
ORA_API void ora_update_at(const double phi[4], const double vel[4], const double g[4], double dt, int zero_v,
                           double phi_out[4], double vel_out[4])
{
    double gp = dot4(g, phi), F[4], p[4], v[4];
    for (int A = 0; A < 4; A++) {
        F[A] = -(g[A] - gp * phi[A]);
        p[A] = phi[A];
        v[A] = zero_v ? 0.0 : vel[A];
    }
    kick_drift(p, v, F, dt);
    for (int A = 0; A < 4; A++) {
        phi_out[A] = p[A];
        vel_out[A] = v[A];
    }
}

/* Power of the velocity field against the force, h^3 sum over I of F . v with
 * F = -gT (the rate dE/dt = -F . v along the flow; Sec. 3, arrest read as
 * "the energy starts to rise"). */
ORA_API double ora_power(const int n[3], double h, const double *gT, const double *vel)
{
    const size_t N3 = n_sites(n);
    double P = 0.0;
    for (int x = 2; x <= n[0] - 3; x++)
        for (int y = 2; y <= n[1] - 3; y++)
            for (int z = 2; z <= n[2] - 3; z++) {
                size_t s = site(n, x, y, z);
                for (int A = 0; A < 4; A++) P += -FLD(gT, A, s) * FLD(vel, A, s);
            }
    return h * h * h * P;
}

/*
 * Run the flow from the state st until st->steps reaches target_steps, the
 * largest tangential gradient falls below tol, or a value stops being finite.
 * At step n:  E_n = E(phi_n); F_n = -(g - (g.phi) phi);
 *             arrest (v_n := 0) if E_n > E_{n-1}            (arrest = 1, energy rule)
 *                            or if h^3 sum F_n . v_n < 0    (arrest = 2, power rule);
 *             stop if max|F_n| < tol;
 *             v_{n+1} = v_n + dt F_n; phi_{n+1} = normalise(phi_n + dt v_{n+1}).
 * arrest = 0 gives the plain Newton flow (no resets); arrest = 3 the gradient
 * flow (Sec. 7.5, the program's flow modes): phi_{n+1} = normalise(phi_n + dt F_n),
 * the velocity stays zero.
 * E_trace / arrest_trace (nullable) receive E_n and the reset flag for each
 * evaluated step, indexed from the step count on entry.
 * Returns the number of evaluated steps.
 */
ORA_API void ora_gradient_literal(const int n[3], double h, const double *mass, const double *phi, double *g);

ORA_API int64_t ora_anf(const int n[3], double h, const double *mass, double dt, double tol, int64_t target_steps, int arrest,
                        int printed, double *phi, double *vel, ora_anf_state *st, double *E_trace, int32_t *arrest_trace)
{
    const size_t N3 = n_sites(n);
    double *g = malloc(4 * N3 * sizeof(double));
    double *gT = malloc(4 * N3 * sizeof(double));
    int64_t evaluated = 0;
    while (st->steps < target_steps) {
        double E = ora_energy(n, h, mass, phi);
        if (printed)
            ora_gradient_literal(n, h, mass, phi, g);
        else
            ora_gradient(n, h, mass, phi, g);
        double r = ora_project(n, phi, g, gT);
        int reset = 0;
        if (arrest == 1) reset = E > st->E_prev;
        else if (arrest == 2) reset = ora_power(n, h, gT, vel) < 0.0;
        if (reset) {
            memset(vel, 0, 4 * N3 * sizeof(double));
            st->arrests++;
        }
        st->E = E;
        st->max_force = r;
        if (E_trace) E_trace[evaluated] = E;
        if (arrest_trace) arrest_trace[evaluated] = reset;
        evaluated++;
        if (!isfinite(E) || !isfinite(r)) {
            st->nonfinite = 1;
            break;
        }
        if (r < tol) {
            st->converged = 1;
            break;
        }
#pragma omp parallel for schedule(static)
        for (int x = 2; x <= n[0] - 3; x++)
            for (int y = 2; y <= n[1] - 3; y++)
                for (int z = 2; z <= n[2] - 3; z++) {
                    size_t s = site(n, x, y, z);
                    double p[4], v[4], F[4];
                    for (int A = 0; A < 4; A++) {
                        p[A] = FLD(phi, A, s);
                        v[A] = FLD(vel, A, s);
                        F[A] = -FLD(gT, A, s);
                    }
                    if (arrest == 3) {
                        double q[4], nrm2 = 0.0;
                        for (int A = 0; A < 4; A++) {
                            q[A] = p[A] + dt * F[A];
                            nrm2 += q[A] * q[A];
                        }
                        double nr = sqrt(nrm2);
                        for (int A = 0; A < 4; A++) {
                            p[A] = q[A] / nr;
                            v[A] = 0.0;
                        }
                    } else {
                        kick_drift(p, v, F, dt);
                    }
                    for (int A = 0; A < 4; A++) {
                        FLD(phi, A, s) = p[A];
                        FLD(vel, A, s) = v[A];
                    }
                }
        st->E_prev = E;
        st->steps++;
    }
    free(g);
    free(gT);
    return evaluated;
}

/* ------------------------------------------------------------------------ */
/* Sec. 4: initial data                                                     */
/* ------------------------------------------------------------------------ */

/* One constituent of a product: a degree-B rational map (B = 1 is the
 * hedgehog R = z) with profile f(r) = prof_a * exp(-r / prof_lambda), centred
 * at X, isorotated by the unit quaternion q = (q0, q1, q2, q3) and turned in
 * space by the rotation D(orient) about X (Sec. 5.3: U(r) -> U(D^-1 r));
 * orient = 0 means unturned. */
typedef struct {
    int32_t degree;      /* polynomial degree of p and q */
    int32_t _pad;
    double p[9][2];      /* coefficients of z^k, k = 0..degree (re, im) */
    double q[9][2];
    double X[3];
    double quat[4];
    double prof_a, prof_lambda;
    double orient[4];
} ora_constituent;

/* Sec. 4.1: unit vector n_R for R = p/q at the direction of x, in homogeneous
 * form.  The point z = tan(theta/2) e^{i phi} of the Riemann sphere is written
 * z = u / w with two charts: u = x1 + i x2, w = r + x3 on the upper half
 * (x3 >= 0), and u = r - x3, w = x1 - i x2 on the lower half, which reaches the
 * south pole z = infinity (u = 2r, w = 0) where the first chart gives 0/0.
 * With P(u,w) = sum p_k u^k w^(B-k) and Q likewise,
 *   n_R = (2 Re(P conj Q), 2 Im(P conj Q), |Q|^2 - |P|^2) / (|P|^2 + |Q|^2),
 * which is (2 Re R, 2 Im R, 1 - |R|^2)/(1 + |R|^2) multiplied through by |Q|^2
 * (a common factor of (u, w) cancels).  At x = 0 the direction is undefined;
 * the north pole's is taken (the profile there gives f = prof_a). */
static void cpow_mul(double *re, double *im, double br, double bi, int e)
{
    for (int k = 0; k < e; k++) {
        double nr = *re * br - *im * bi, ni = *re * bi + *im * br;
        *re = nr;
        *im = ni;
    }
}

static void rational_map_direction(const ora_constituent *c, const double x_in[3], double nhat[3])
{
    double x[3] = {x_in[0], x_in[1], x_in[2]};
    double r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    if (r == 0.0) {
        x[2] = 1.0;
        r = 1.0;
    }
    double ur, ui, wr, wi;
    if (x[2] >= 0.0) {
        ur = x[0];
        ui = x[1];
        wr = r + x[2];
        wi = 0.0;
    } else {
        ur = r - x[2];
        ui = 0.0;
        wr = x[0];
        wi = -x[1];
    }
    double Pr = 0, Pi = 0, Qr = 0, Qi = 0;
    for (int k = 0; k <= c->degree; k++) {
        /* u^k w^(B-k) */
        double tr = 1.0, ti = 0.0;
        cpow_mul(&tr, &ti, ur, ui, k);
        cpow_mul(&tr, &ti, wr, wi, c->degree - k);
        Pr += c->p[k][0] * tr - c->p[k][1] * ti;
        Pi += c->p[k][0] * ti + c->p[k][1] * tr;
        Qr += c->q[k][0] * tr - c->q[k][1] * ti;
        Qi += c->q[k][0] * ti + c->q[k][1] * tr;
    }
    /* P conj(Q) */
    double cr = Pr * Qr + Pi * Qi, ci = Pi * Qr - Pr * Qi;
    double p2 = Pr * Pr + Pi * Pi, q2 = Qr * Qr + Qi * Qi;
    double den = p2 + q2;
    nhat[0] = 2.0 * cr / den;
    nhat[1] = 2.0 * ci / den;
    nhat[2] = (q2 - p2) / den;
}

/* Sec. 5.3: A (x.tau) A^dagger = (D(A) x).tau with
 * D(A) x = (a0^2 - |a|^2) x + 2 (a.x) a - 2 a0 (a cross x). */
static void isorotate(const double qa[4], const double v[3], double out[3])
{
    double a0 = qa[0], a[3] = {qa[1], qa[2], qa[3]};
    double aa = a[0] * a[0] + a[1] * a[1] + a[2] * a[2];
    double ax = a[0] * v[0] + a[1] * v[1] + a[2] * v[2];
    double cr[3] = {a[1] * v[2] - a[2] * v[1], a[2] * v[0] - a[0] * v[2], a[0] * v[1] - a[1] * v[0]};
    for (int k = 0; k < 3; k++) out[k] = (a0 * a0 - aa) * v[k] + 2.0 * ax * a[k] - 2.0 * a0 * cr[k];
}

/* U = phi0 + i phi.tau ; (a0 + i a.tau)(b0 + i b.tau) = (a0 b0 - a.b) + i (a0 b + b0 a - a x b).tau */
static void su2_mul(const double a[4], const double b[4], double out[4])
{
    double o0 = a[0] * b[0] - (a[1] * b[1] + a[2] * b[2] + a[3] * b[3]);
    double cx = a[2] * b[3] - a[3] * b[2], cy = a[3] * b[1] - a[1] * b[3], cz = a[1] * b[2] - a[2] * b[1];
    out[1] = a[0] * b[1] + b[0] * a[1] - cx;
    out[2] = a[0] * b[2] + b[0] * a[2] - cy;
    out[3] = a[0] * b[3] + b[0] * a[3] - cz;
    out[0] = o0;
}

/* Field of one constituent at position x: U_k = A exp(i f n_R.tau) A^dagger at x - X. */
static void constituent_field(const ora_constituent *c, const double x[3], double U[4])
{
    double d[3] = {x[0] - c->X[0], x[1] - c->X[1], x[2] - c->X[2]};
    if (c->orient[0] != 0.0 || c->orient[1] != 0.0 || c->orient[2] != 0.0 || c->orient[3] != 0.0) {
        /* D(B)^-1 = D(B^dagger), B^dagger = (b0, -b) */
        double binv[4] = {c->orient[0], -c->orient[1], -c->orient[2], -c->orient[3]}, dd[3];
        isorotate(binv, d, dd);
        d[0] = dd[0];
        d[1] = dd[1];
        d[2] = dd[2];
    }
    double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double f = c->prof_a * exp(-r / c->prof_lambda);
    double nhat[3], rot[3];
    rational_map_direction(c, d, nhat);
    isorotate(c->quat, nhat, rot);
    double sf = sin(f);
    U[0] = cos(f);
    U[1] = sf * rot[0];
    U[2] = sf * rot[1];
    U[3] = sf * rot[2];
}

/* Sec. 4.2: U = prod_{k=1..N} A_k U_k(x - X_k) A_k^dagger, taken left to
 * right; interior sites only, the two outer layers per face set to vacuum. */
ORA_API void ora_init_product(const int n[3], double h, int32_t nc, const ora_constituent *c, double *phi)
{
    const size_t N3 = n_sites(n);
#pragma omp parallel for schedule(static)
    for (int ix = 0; ix < n[0]; ix++)
        for (int iy = 0; iy < n[1]; iy++)
            for (int iz = 0; iz < n[2]; iz++) {
                size_t s = site(n, ix, iy, iz);
                double U[4] = {1.0, 0.0, 0.0, 0.0};
                if (interior(n, ix, iy, iz)) {
                    double x[3] = {(ix - 0.5 * (n[0] - 1)) * h, (iy - 0.5 * (n[1] - 1)) * h,
                                   (iz - 0.5 * (n[2] - 1)) * h};
                    for (int k = 0; k < nc; k++) {
                        double Uk[4], t[4];
                        constituent_field(&c[k], x, Uk);
                        su2_mul(U, Uk, t);
                        memcpy(U, t, sizeof U);
                    }
                }
                for (int A = 0; A < 4; A++) FLD(phi, A, s) = U[A];
            }
}

/* ------------------------------------------------------------------------ */
/* random constituents (smorgasbord-style initial data, Sec. 4.2)           */
/* ------------------------------------------------------------------------ */

/* SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): the k-th output is the
 * finaliser applied to seed + k * 0x9E3779B97F4A7C15. */
typedef struct {
    uint64_t state;
} ora_splitmix;

static uint64_t splitmix_next(ora_splitmix *g)
{
    g->state += 0x9E3779B97F4A7C15ULL;
    uint64_t z = g->state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* uniform in [0, 1) from the top 53 bits */
static double splitmix_uniform(ora_splitmix *g) { return (double)(splitmix_next(g) >> 11) * 0x1.0p-53; }

ORA_API uint64_t ora_splitmix64(uint64_t seed, int64_t k)
{
    ora_splitmix g = {seed};
    uint64_t v = 0;
    for (int64_t i = 0; i <= k; i++) v = splitmix_next(&g);
    return v;
}

/* B unit-charge constituents (hedgehogs) with centres uniform in the ball of
 * the given radius (rejection from the enclosing cube) and Haar-random
 * isorotations (Shoemake, Graphics Gems III, 1992):
 *   q = (sqrt(1-u1) sin 2pi u2, sqrt(1-u1) cos 2pi u2, sqrt(u1) sin 2pi u3, sqrt(u1) cos 2pi u3).
 * Draw order per constituent: centre attempts (3 uniforms each), then u1, u2, u3. */
ORA_API void ora_random_constituents(uint64_t seed, int32_t B, double radius, double prof_a, double prof_lambda,
                                     ora_constituent *out)
{
    ora_splitmix g = {seed};
    for (int k = 0; k < B; k++) {
        ora_constituent *c = &out[k];
        memset(c, 0, sizeof *c);
        c->degree = 1;
        c->p[1][0] = 1.0; /* p = z */
        c->q[0][0] = 1.0; /* q = 1 */
        for (;;) {
            double X0 = radius * (2.0 * splitmix_uniform(&g) - 1.0);
            double X1 = radius * (2.0 * splitmix_uniform(&g) - 1.0);
            double X2 = radius * (2.0 * splitmix_uniform(&g) - 1.0);
            if (X0 * X0 + X1 * X1 + X2 * X2 <= radius * radius) {
                c->X[0] = X0;
                c->X[1] = X1;
                c->X[2] = X2;
                break;
            }
        }
        double u1 = splitmix_uniform(&g), u2 = splitmix_uniform(&g), u3 = splitmix_uniform(&g);
        double s1 = sqrt(1.0 - u1), s2 = sqrt(u1);
        c->quat[0] = s1 * sin(2.0 * M_PI * u2);
        c->quat[1] = s1 * cos(2.0 * M_PI * u2);
        c->quat[2] = s2 * sin(2.0 * M_PI * u3);
        c->quat[3] = s2 * cos(2.0 * M_PI * u3);
        c->prof_a = prof_a;
        c->prof_lambda = prof_lambda;
    }
}

/* ------------------------------------------------------------------------ */
/* the paper-literal Euler-Lagrange expression (eq. Sigma model EL         */
/* equations, halved), evaluated with the five-point second derivative and */
/* the mixed derivatives D_i D_j (the product of two first-difference      */
/* stencils, Sec. 3), on every interior site; the frozen layers supply the */
/* values the stencils reach.  The program's form of the force (the        */
/* library's optional printed-form flow).                                  */
/* ------------------------------------------------------------------------ */

ORA_API void ora_gradient_literal(const int n[3], double h, const double *mass, const double *phi, double *g)
{
    const size_t N3 = n_sites(n);
    /* a_i on every site whose i-th coordinate admits the stencil (2 .. n_i - 3),
     * whatever its other coordinates: D_j D_i at an interior site reads a_i at
     * distance <= 2 along j only */
    double *a = malloc(12 * N3 * sizeof(double));
    memset(a, 0, 12 * N3 * sizeof(double));
#pragma omp parallel for schedule(static)
    for (int x = 0; x < n[0]; x++)
        for (int y = 0; y < n[1]; y++)
            for (int z = 0; z < n[2]; z++) {
                const int c[3] = {x, y, z};
                size_t s = site(n, x, y, z);
                for (int i = 0; i < 3; i++) {
                    if (c[i] < 2 || c[i] > n[i] - 3) continue;
                    for (int A = 0; A < 4; A++)
                        a[((size_t)i * 4 + A) * N3 + s] = d1(phi + (size_t)A * N3, n, i, x, y, z, h);
                }
            }
    memset(g, 0, 4 * N3 * sizeof(double));
#pragma omp parallel for schedule(static)
    for (int x = 2; x <= n[0] - 3; x++)
        for (int y = 2; y <= n[1] - 3; y++)
            for (int z = 2; z <= n[2] - 3; z++) {
                size_t s = site(n, x, y, z);
                double d[3][4], dd[3][3][4];
                for (int i = 0; i < 3; i++)
                    for (int A = 0; A < 4; A++) d[i][A] = a[((size_t)i * 4 + A) * N3 + s];
                for (int i = 0; i < 3; i++)
                    for (int j = 0; j < 3; j++)
                        for (int A = 0; A < 4; A++) {
                            if (i == j)
                                dd[i][j][A] = d2(phi + (size_t)A * N3, n, i, x, y, z, h);
                            else
                                dd[i][j][A] = d1(a + ((size_t)j * 4 + A) * N3, n, i, x, y, z, h);
                        }
                double S = 0.0;
                for (int j = 0; j < 3; j++) S += dot4(d[j], d[j]);
                for (int A = 0; A < 4; A++) {
                    double t = 0.0;
                    for (int i = 0; i < 3; i++) {
                        t += dd[i][i][A] * (1.0 + S);
                        double c = 0.0;
                        for (int j = 0; j < 3; j++) c += dot4(dd[i][j], d[j]) - dot4(dd[j][j], d[i]);
                        t += d[i][A] * c;
                        for (int j = 0; j < 3; j++) t -= dd[i][j][A] * dot4(d[i], d[j]);
                    }
                    g[(size_t)A * N3 + s] = -t + (A == 0 ? potential_slope(mass, phi[s]) : 0.0);
                }
            }
    free(a);
}

ORA_API int ora_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

ORA_API void ora_set_num_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}
