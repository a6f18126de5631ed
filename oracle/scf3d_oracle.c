/*
 * FP64 CPU oracle of the binary Shan-Chen model on a three-dimensional D3Q19 lattice: the 3-D
 * capillary that S. Chibbaro's "Capillary filling with pseudo-potential binary Lattice-Boltzmann
 * model" names as future work (Conclusions).  TEST INFRASTRUCTURE ONLY, like scf_oracle.c: the
 * tests load it; the product path never does, and it shares no code with the HIP library.
 *
 * The step is the one of Sec. 2 (eqs. lbe, feq, forcing, forcingw, the common velocity U and the
 * shifted equilibrium velocity), written for D3Q19:
 *  - equilibrium f_i^eq = w_i n (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u) with w = 1/3 (rest),
 *    1/18 (6 axis links), 1/36 (12 edge links);
 *  - bulk force F_k = -n_k G sum_{i>0} w_i n_kbar(x + c_i) c_i, wall force
 *    F_k += -n_k G_kw sum_{i>0} w_i s(x + c_i) c_i, with psi = n and psi = 0 on solid nodes;
 *  - U = sum_k (m_k j_k / tau_k) / sum_k (m_k n_k / tau_k); u_k^eq = U + tau_k F_k / (m_k n_k);
 *  - BGK relaxation, then streaming with half-way bounce-back at solid nodes.
 * The z-projection of these weights is the D2Q9 set with rest fraction 4/9, so a state that does
 * not depend on z evolves exactly as the two-dimensional model.
 *
 * Geometry: nx x ny x nz, periodic in all three directions; solid nodes are those with
 * x in [x0, x1) and (y == 0 or y == ny-1) [walls_y], or (z == 0 or z == nz-1) [walls_z].
 */
#include "scf_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <omp.h>

/* D3Q19: rest, six axis links, twelve edge links. */
static const int CX3[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int CY3[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int CZ3[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
static const double W3[19] = {1.0 / 3,  1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                              1.0 / 18, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                              1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                              1.0 / 36};

struct orc3 {
    int nx, ny, nz, x0, x1, walls_y, walls_z;
    double G, gw[2], tau[2], mass[2];
    int64_t t;
    double* f;    /* [2][19][nz][ny][nx] */
    double* fs;   /* post-collision */
    double* n;    /* [2][nz][ny][nx] */
};

static int opp3(int i) {
    for (int j = 0; j < 19; ++j)
        if (CX3[j] == -CX3[i] && CY3[j] == -CY3[i] && CZ3[j] == -CZ3[i]) return j;
    return 0;
}

#define F3(s, k, i, z, y, x) \
    (((((size_t)(k) * 19 + (i)) * (size_t)(s)->nz + (z)) * (size_t)(s)->ny + (y)) * (size_t)(s)->nx + (x))
#define N3(s, k, z, y, x) ((((size_t)(k) * (s)->nz + (z)) * (size_t)(s)->ny + (y)) * (size_t)(s)->nx + (x))

static int wrap(int v, int n) { return ((v % n) + n) % n; }

static int solid3(const orc3_t* s, int x, int y, int z) {
    if (x < s->x0 || x >= s->x1) return 0;
    if (s->walls_y && (y == 0 || y == s->ny - 1)) return 1;
    if (s->walls_z && (z == 0 || z == s->nz - 1)) return 1;
    return 0;
}

orc3_t* orc3_create(int nx, int ny, int nz, int x0, int x1, int walls_y, int walls_z, double G,
                    const double gw[2], const double tau[2], const double mass[2]) {
    if (nx < 1 || ny < 1 || nz < 1) return NULL;
    orc3_t* s = (orc3_t*)calloc(1, sizeof(orc3_t));
    s->nx = nx; s->ny = ny; s->nz = nz; s->x0 = x0; s->x1 = x1;
    s->walls_y = walls_y; s->walls_z = walls_z;
    s->G = G;
    for (int k = 0; k < 2; ++k) { s->gw[k] = gw[k]; s->tau[k] = tau[k]; s->mass[k] = mass[k]; }
    size_t cells = (size_t)nx * ny * nz;
    s->f = (double*)calloc(2 * 19 * cells, sizeof(double));
    s->fs = (double*)calloc(2 * 19 * cells, sizeof(double));
    s->n = (double*)calloc(2 * cells, sizeof(double));
    return s;
}

void orc3_destroy(orc3_t* s) {
    if (!s) return;
    free(s->f); free(s->fs); free(s->n); free(s);
}

int64_t orc3_time(const orc3_t* s) { return s->t; }

/* The D3Q19 equilibrium for one node. */
void orc3_feq(double n, double ux, double uy, double uz, double out[19]) {
    double uu = ux * ux + uy * uy + uz * uz;
    for (int i = 0; i < 19; ++i) {
        double cu = CX3[i] * ux + CY3[i] * uy + CZ3[i] * uz;
        out[i] = W3[i] * n * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    }
}

/* rho arrays are nz*ny*nx (x fastest); populations at rest, solid nodes zero. */
void orc3_init(orc3_t* s, const double* rhoA, const double* rhoB) {
    const double* rho[2] = {rhoA, rhoB};
    double fe[19];
    for (int k = 0; k < 2; ++k)
        for (int z = 0; z < s->nz; ++z)
            for (int y = 0; y < s->ny; ++y)
                for (int x = 0; x < s->nx; ++x) {
                    int sol = solid3(s, x, y, z);
                    size_t c = ((size_t)z * s->ny + y) * s->nx + x;
                    orc3_feq(sol ? 0.0 : rho[k][c] / s->mass[k], 0.0, 0.0, 0.0, fe);
                    for (int i = 0; i < 19; ++i) s->f[F3(s, k, i, z, y, x)] = sol ? 0.0 : fe[i];
                }
    s->t = 0;
}

static void density3(orc3_t* s) {
    for (int k = 0; k < 2; ++k)
        for (int z = 0; z < s->nz; ++z)
            for (int y = 0; y < s->ny; ++y)
                for (int x = 0; x < s->nx; ++x) {
                    double v = 0.0;
                    if (!solid3(s, x, y, z))
                        for (int i = 0; i < 19; ++i) v += s->f[F3(s, k, i, z, y, x)];
                    s->n[N3(s, k, z, y, x)] = v;
                }
}

static void collide3(orc3_t* s) {
    density3(s);
#pragma omp parallel for collapse(2) num_threads(orc_threads())
    for (int z = 0; z < s->nz; ++z)
        for (int y = 0; y < s->ny; ++y)
            for (int x = 0; x < s->nx; ++x) {
                if (solid3(s, x, y, z)) {
                    for (int k = 0; k < 2; ++k)
                        for (int i = 0; i < 19; ++i) s->fs[F3(s, k, i, z, y, x)] = 0.0;
                    continue;
                }
                double nk[2], j[2][3], F[2][3] = {{0, 0, 0}, {0, 0, 0}};
                for (int k = 0; k < 2; ++k) {
                    nk[k] = s->n[N3(s, k, z, y, x)];
                    j[k][0] = j[k][1] = j[k][2] = 0.0;
                    for (int i = 0; i < 19; ++i) {
                        double v = s->f[F3(s, k, i, z, y, x)];
                        j[k][0] += CX3[i] * v; j[k][1] += CY3[i] * v; j[k][2] += CZ3[i] * v;
                    }
                }
                /* eq. forcing and eq. forcingw on the D3Q19 neighbours */
                for (int i = 1; i < 19; ++i) {
                    int xn = wrap(x + CX3[i], s->nx), yn = wrap(y + CY3[i], s->ny), zn = wrap(z + CZ3[i], s->nz);
                    double sw = solid3(s, xn, yn, zn) ? 1.0 : 0.0;
                    for (int k = 0; k < 2; ++k) {
                        double psib = s->n[N3(s, 1 - k, zn, yn, xn)];
                        double a = -nk[k] * W3[i] * (s->G * psib + s->gw[k] * sw);
                        F[k][0] += a * CX3[i]; F[k][1] += a * CY3[i]; F[k][2] += a * CZ3[i];
                    }
                }
                double num[3] = {0, 0, 0}, den = 0.0;
                for (int k = 0; k < 2; ++k) {
                    for (int d = 0; d < 3; ++d) num[d] += s->mass[k] * j[k][d] / s->tau[k];
                    den += s->mass[k] * nk[k] / s->tau[k];
                }
                for (int k = 0; k < 2; ++k) {
                    double rho = s->mass[k] * nk[k];
                    double u[3];
                    for (int d = 0; d < 3; ++d) u[d] = num[d] / den + s->tau[k] * F[k][d] / rho;
                    double fe[19];
                    orc3_feq(nk[k], u[0], u[1], u[2], fe);
                    for (int i = 0; i < 19; ++i) {
                        double v = s->f[F3(s, k, i, z, y, x)];
                        s->fs[F3(s, k, i, z, y, x)] = v - (v - fe[i]) / s->tau[k];
                    }
                }
            }
}

static void stream3(orc3_t* s) {
#pragma omp parallel for collapse(2) num_threads(orc_threads())
    for (int z = 0; z < s->nz; ++z)
        for (int y = 0; y < s->ny; ++y)
            for (int x = 0; x < s->nx; ++x) {
                int sol = solid3(s, x, y, z);
                for (int k = 0; k < 2; ++k)
                    for (int i = 0; i < 19; ++i) {
                        double v = 0.0;
                        if (!sol) {
                            int xs = wrap(x - CX3[i], s->nx), ys = wrap(y - CY3[i], s->ny),
                                zs = wrap(z - CZ3[i], s->nz);
                            v = solid3(s, xs, ys, zs) ? s->fs[F3(s, k, opp3(i), z, y, x)]
                                                      : s->fs[F3(s, k, i, zs, ys, xs)];
                        }
                        s->f[F3(s, k, i, z, y, x)] = v;
                    }
            }
    s->t += 1;
}

void orc3_step(orc3_t* s, int64_t nsteps) {
    for (int64_t i = 0; i < nsteps; ++i) {
        collide3(s);
        stream3(s);
    }
}

void orc3_density(orc3_t* s, double* nA, double* nB) {
    density3(s);
    size_t cells = (size_t)s->nx * s->ny * s->nz;
    memcpy(nA, s->n, cells * sizeof(double));
    memcpy(nB, s->n + cells, cells * sizeof(double));
}

void orc3_get_f(const orc3_t* s, double* f) {
    memcpy(f, s->f, (size_t)2 * 19 * s->nx * s->ny * s->nz * sizeof(double));
}

void orc3_set_f(orc3_t* s, const double* f) {
    memcpy(s->f, f, (size_t)2 * 19 * s->nx * s->ny * s->nz * sizeof(double));
}

/* Mass per component and the centre-line front: on the line y = (ny-1)/2, z = (nz-1)/2
 * (averaged over the two or four nearest lines for even sizes), phi = n_A - n_B, first
 * downward crossing scanning from x0/2, linearly refined, relative to x0. */
void orc3_observe(orc3_t* s, double mass[2], double* z_front) {
    density3(s);
    for (int k = 0; k < 2; ++k) {
        double m = 0.0;
        for (int z = 0; z < s->nz; ++z)
            for (int y = 0; y < s->ny; ++y)
                for (int x = 0; x < s->nx; ++x) m += s->n[N3(s, k, z, y, x)];
        mass[k] = m;
    }
    int ya = (s->ny - 1) / 2, yb = s->ny / 2, za = (s->nz - 1) / 2, zb = s->nz / 2;
    *z_front = NAN;
    double prev = 0.0;
    for (int x = s->x0 / 2; x < s->nx; ++x) {
        double phi = 0.0;
        int ys[2] = {ya, yb}, zs[2] = {za, zb};
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                phi += 0.25 * (s->n[N3(s, 0, zs[b], ys[a], x)] - s->n[N3(s, 1, zs[b], ys[a], x)]);
        if (x > s->x0 / 2 && prev >= 0.0 && phi < 0.0) {
            *z_front = (double)(x - 1) + prev / (prev - phi) - s->x0;
            return;
        }
        prev = phi;
    }
}
