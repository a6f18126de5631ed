/*
 * FP64 CPU oracle of the binary Shan-Chen lattice Boltzmann model (S. Chibbaro,
 * "Capillary filling with pseudo-potential binary Lattice-Boltzmann model", Sec. 2-3).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the CPU-baseline leg
 * of the bench, never by the product path.  It shares no code with the HIP library.
 *
 * Plain per-node loops, FP64, built with -ffp-contract=off so runs are reproducible.  The
 * OpenMP pragmas only split the independent per-node loops over rows; every node's
 * arithmetic is the same whatever the thread count.
 *
 * Readings of points the paper leaves open (each also listed in the design notes):
 *  - force weights: the bulk and wall neighbour sums use the D2Q9 weights 1/9 (|x'-x| = 1)
 *    and 1/36 (|x'-x| = sqrt 2) times a coupling G.  This is the paper's interaction matrix
 *    (g on axis, g/4 on diagonals) with g = G/9.
 *  - psi_k = n_k in the fluid and 0 on solid nodes; walls act only through eq. forcingw.
 *  - eq. forcingw uses the same eight neighbours and weights, with rho_w folded into G_kw.
 *  - the sum defining U runs over components.
 *  - bounce-back is the half-way (link) rule: a population that would come from a solid node
 *    is the node's own post-collision population of the opposite direction.
 *  - forces use the densities of the state before collision (time t).
 */
#include "scf_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* D2Q9 velocities as numbered in Sec. 2: c_0 = 0; c_1..c_4 = (cos, sin) of (i-1)*90 deg;
 * c_5..c_8 = sqrt 2 (cos, sin) of 45 + (i-5)*90 deg. */
static const int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
/* Interaction weights per neighbour (eq. forcing matrix shape g, g/4, normalised as D2Q9). */
static const double WF[9] = {0.0, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                             1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

struct orc {
    int nx, ny, x0, x1, periodic_x;
    double G, gw[2], tau[2], alpha[2], mass[2];
    int64_t t;
    double* f;     /* [2][9][ny][nx] state f(x, t) */
    double* fs;    /* [2][9][ny][nx] post-collision f*(x, t) */
    double* n;     /* [2][ny][nx] densities of the current state (scratch) */
    unsigned char* mask;   /* optional [ny][nx] solid mask (non-zero = solid), replaces the rows */
};

static int g_threads = 1;

void orc_set_threads(int nthreads) { g_threads = nthreads > 0 ? nthreads : 1; }
int orc_threads(void) { return g_threads; }

#define FIDX(s, k, i, y, x) ((((size_t)(k) * 9 + (i)) * (size_t)(s)->ny + (y)) * (size_t)(s)->nx + (x))
#define NIDX(s, k, y, x) (((size_t)(k) * (s)->ny + (y)) * (size_t)(s)->nx + (x))

static int is_solid(const orc_t* s, int x, int y) {
    if (s->mask) return s->mask[(size_t)y * s->nx + x] != 0;
    return (y == 0 || y == s->ny - 1) && x >= s->x0 && x < s->x1;
}

/* Neighbour coordinates with periodic wrap in y, and in x unless periodic_x is 0
 * (then x is clamped to the box: only used to evolve an inner window of a larger box). */
static int wrap_x(const orc_t* s, int x) {
    if (s->periodic_x) return ((x % s->nx) + s->nx) % s->nx;
    return x < 0 ? 0 : (x >= s->nx ? s->nx - 1 : x);
}
static int wrap_y(const orc_t* s, int y) { return ((y % s->ny) + s->ny) % s->ny; }

orc_t* orc_create(int nx, int ny, int x0, int x1, int periodic_x, double G, const double gw[2],
                  const double tau[2], const double alpha[2], const double mass[2]) {
    if (nx < 1 || ny < 1) return NULL;
    orc_t* s = (orc_t*)calloc(1, sizeof(orc_t));
    s->nx = nx; s->ny = ny; s->x0 = x0; s->x1 = x1; s->periodic_x = periodic_x;
    s->G = G;
    for (int k = 0; k < 2; ++k) {
        s->gw[k] = gw[k]; s->tau[k] = tau[k]; s->alpha[k] = alpha[k]; s->mass[k] = mass[k];
    }
    size_t nf = (size_t)2 * 9 * ny * nx;
    s->f = (double*)calloc(nf, sizeof(double));
    s->fs = (double*)calloc(nf, sizeof(double));
    s->n = (double*)calloc((size_t)2 * ny * nx, sizeof(double));
    return s;
}

void orc_destroy(orc_t* s) {
    if (!s) return;
    free(s->f); free(s->fs); free(s->n); free(s->mask); free(s);
}

void orc_set_mask(orc_t* s, const unsigned char* mask) {
    free(s->mask);
    s->mask = NULL;
    if (!mask) return;
    s->mask = (unsigned char*)malloc((size_t)s->ny * s->nx);
    memcpy(s->mask, mask, (size_t)s->ny * s->nx);
}

int64_t orc_time(const orc_t* s) { return s->t; }

/* eqs. feq1-feq3: the equilibrium with rest fraction alpha for density n and velocity u. */
void orc_feq(double n, double ux, double uy, double alpha, double out[9]) {
    double uu = ux * ux + uy * uy;
    out[0] = alpha * n - (2.0 / 3.0) * n * uu;
    for (int i = 1; i <= 4; ++i) {
        double cu = CX[i] * ux + CY[i] * uy;
        out[i] = (1.0 - alpha) * n / 5.0 + (1.0 / 3.0) * n * cu + 0.5 * n * cu * cu
                 - (1.0 / 6.0) * n * uu;
    }
    for (int i = 5; i <= 8; ++i) {
        double cu = CX[i] * ux + CY[i] * uy;
        out[i] = (1.0 - alpha) * n / 20.0 + (1.0 / 12.0) * n * cu + 0.125 * n * cu * cu
                 - (1.0 / 24.0) * n * uu;
    }
}

void orc_init(orc_t* s, const double* rhoA, const double* rhoB) {
    const double* rho[2] = {rhoA, rhoB};
    double fe[9];
    for (int k = 0; k < 2; ++k)
        for (int y = 0; y < s->ny; ++y)
            for (int x = 0; x < s->nx; ++x) {
                int solid = is_solid(s, x, y);
                /* n_k = rho_k / m_k; populations at rest */
                double nk = solid ? 0.0 : rho[k][(size_t)y * s->nx + x] / s->mass[k];
                orc_feq(nk, 0.0, 0.0, s->alpha[k], fe);
                for (int i = 0; i < 9; ++i) s->f[FIDX(s, k, i, y, x)] = solid ? 0.0 : fe[i];
            }
    s->t = 0;
}

/* n_k = sum_i f^k_i on fluid nodes, 0 on solid nodes (psi = 0 in the wall). */
static void compute_density(orc_t* s) {
    #pragma omp parallel for num_threads(g_threads) schedule(static)
    for (int y = 0; y < s->ny; ++y)
        for (int x = 0; x < s->nx; ++x)
            for (int k = 0; k < 2; ++k) {
                double nk = 0.0;
                if (!is_solid(s, x, y))
                    for (int i = 0; i < 9; ++i) nk += s->f[FIDX(s, k, i, y, x)];
                s->n[NIDX(s, k, y, x)] = nk;
            }
}

/* Everything the collision at one fluid node needs (Sec. 2), from the densities in s->n. */
typedef struct {
    double n[2], j[2][2], F[2][2], U[2], ueq[2][2];
} node_state;

static void node_macro(const orc_t* s, int x, int y, node_state* o) {
    /* densities and momenta: n_k = sum_i f_i, j_k = sum_i c_i f_i (rho_k u_k = m_k j_k) */
    for (int k = 0; k < 2; ++k) {
        o->n[k] = s->n[NIDX(s, k, y, x)];
        double jx = 0.0, jy = 0.0;
        for (int i = 0; i < 9; ++i) {
            double fi = s->f[FIDX(s, k, i, y, x)];
            jx += CX[i] * fi;
            jy += CY[i] * fi;
        }
        o->j[k][0] = jx; o->j[k][1] = jy;
    }
    /* eq. forcing with psi = n and G_{k kbar} = G w_i between different components only:
     *   F_1k(x) = -psi_k(x) sum_{x'} G_{k kbar} psi_kbar(x') (x' - x)
     * eq. forcingw with the same neighbours, s(x') = 1 on solid nodes:
     *   F_2k(x) = -n_k(x) sum_{x'} G_kw s(x') (x' - x)                                  */
    for (int k = 0; k < 2; ++k) {
        int kb = 1 - k;
        double sbx = 0.0, sby = 0.0, swx = 0.0, swy = 0.0;
        for (int i = 1; i < 9; ++i) {
            int xn = wrap_x(s, x + CX[i]);
            int yn = wrap_y(s, y + CY[i]);
            double psi_kb = s->n[NIDX(s, kb, yn, xn)];   /* 0 on solid nodes */
            sbx += WF[i] * psi_kb * CX[i];
            sby += WF[i] * psi_kb * CY[i];
            double sw = is_solid(s, xn, yn) ? 1.0 : 0.0;
            swx += WF[i] * sw * CX[i];
            swy += WF[i] * sw * CY[i];
        }
        double psi_k = o->n[k];
        o->F[k][0] = -psi_k * s->G * sbx - o->n[k] * s->gw[k] * swx;
        o->F[k][1] = -psi_k * s->G * sby - o->n[k] * s->gw[k] * swy;
    }
    /* common velocity: U = sum_k (rho_k u_k / tau_k) / sum_k (rho_k / tau_k) */
    double num[2] = {0.0, 0.0}, den = 0.0;
    for (int k = 0; k < 2; ++k) {
        double rho_k = s->mass[k] * o->n[k];
        num[0] += s->mass[k] * o->j[k][0] / s->tau[k];
        num[1] += s->mass[k] * o->j[k][1] / s->tau[k];
        den += rho_k / s->tau[k];
    }
    o->U[0] = num[0] / den;
    o->U[1] = num[1] / den;
    /* shifted equilibrium velocity: rho_k u_k^eq = rho_k U + tau_k F_k */
    for (int k = 0; k < 2; ++k) {
        double rho_k = s->mass[k] * o->n[k];
        o->ueq[k][0] = o->U[0] + s->tau[k] * o->F[k][0] / rho_k;
        o->ueq[k][1] = o->U[1] + s->tau[k] * o->F[k][1] / rho_k;
    }
}

void orc_collide(orc_t* s) {
    compute_density(s);
    #pragma omp parallel for num_threads(g_threads) schedule(static)
    for (int y = 0; y < s->ny; ++y)
        for (int x = 0; x < s->nx; ++x) {
            if (is_solid(s, x, y)) {
                for (int k = 0; k < 2; ++k)
                    for (int i = 0; i < 9; ++i) s->fs[FIDX(s, k, i, y, x)] = 0.0;
                continue;
            }
            node_state o;
            node_macro(s, x, y, &o);
            for (int k = 0; k < 2; ++k) {
                double fe[9];
                orc_feq(o.n[k], o.ueq[k][0], o.ueq[k][1], s->alpha[k], fe);
                /* eq. lbe: f* = f - (f - f^eq) / tau_k   (Delta t = 1) */
                for (int i = 0; i < 9; ++i) {
                    double fi = s->f[FIDX(s, k, i, y, x)];
                    s->fs[FIDX(s, k, i, y, x)] = fi - (fi - fe[i]) / s->tau[k];
                }
            }
        }
}

void orc_stream(orc_t* s) {
    /* f_i(x, t+1) = f*_i(x - c_i, t), or f*_{opp(i)}(x, t) when x - c_i is solid. */
    #pragma omp parallel for num_threads(g_threads) schedule(static)
    for (int y = 0; y < s->ny; ++y)
        for (int x = 0; x < s->nx; ++x) {
            int solid = is_solid(s, x, y);
            for (int k = 0; k < 2; ++k)
                for (int i = 0; i < 9; ++i) {
                    double v = 0.0;
                    if (!solid) {
                        int xs = wrap_x(s, x - CX[i]);
                        int ys = wrap_y(s, y - CY[i]);
                        v = is_solid(s, xs, ys) ? s->fs[FIDX(s, k, OPP[i], y, x)]
                                                : s->fs[FIDX(s, k, i, ys, xs)];
                    }
                    s->f[FIDX(s, k, i, y, x)] = v;
                }
        }
    s->t += 1;
}

void orc_step(orc_t* s, int64_t nsteps) {
    for (int64_t t = 0; t < nsteps; ++t) {
        orc_collide(s);
        orc_stream(s);
    }
}

void orc_macro(orc_t* s, double* n, double* j, double* F, double* U, double* ueq) {
    compute_density(s);
    size_t plane = (size_t)s->ny * s->nx;
    for (int y = 0; y < s->ny; ++y)
        for (int x = 0; x < s->nx; ++x) {
            size_t p = (size_t)y * s->nx + x;
            node_state o;
            memset(&o, 0, sizeof o);
            if (!is_solid(s, x, y)) node_macro(s, x, y, &o);
            for (int k = 0; k < 2; ++k) {
                if (n) n[k * plane + p] = o.n[k];
                for (int d = 0; d < 2; ++d) {
                    if (j) j[(k * 2 + d) * plane + p] = o.j[k][d];
                    if (F) F[(k * 2 + d) * plane + p] = o.F[k][d];
                    if (ueq) ueq[(k * 2 + d) * plane + p] = o.ueq[k][d];
                }
            }
            if (U) { U[p] = o.U[0]; U[plane + p] = o.U[1]; }
        }
}

void orc_get_f(const orc_t* s, double* f) {
    memcpy(f, s->f, sizeof(double) * 2 * 9 * (size_t)s->ny * s->nx);
}

void orc_set_f(orc_t* s, const double* f) {
    memcpy(s->f, f, sizeof(double) * 2 * 9 * (size_t)s->ny * s->nx);
}

void orc_density(orc_t* s, double* nA, double* nB) {
    compute_density(s);
    size_t plane = (size_t)s->ny * s->nx;
    memcpy(nA, s->n, sizeof(double) * plane);
    memcpy(nB, s->n + plane, sizeof(double) * plane);
}

/* Observables of the filling experiment (Sec. 3): the centre-line front, the precursor film
 * front on the two wall-adjacent rows, the per-component mass and a health flag.
 *  - centre line: phi = n_A - n_B on row ny/2 - 1 and ny/2 averaged (ny even) or row
 *    (ny-1)/2 (ny odd); scanning from the liquid-reservoir centre xs = x0/2, the front is the
 *    first x with phi(x) >= 0 > phi(x+1), refined linearly, reported relative to x0.
 *  - precursor: the first x >= xs on a wall-adjacent row where n_A falls through one third of
 *    its bulk value n_A(xs, centre line), refined linearly, relative to x0. */
static double centre_value(const orc_t* s, int k, int x) {
    const double* nk = s->n + (size_t)k * s->ny * s->nx;
    if (s->ny % 2 == 0)
        return 0.5 * (nk[(size_t)(s->ny / 2 - 1) * s->nx + x] + nk[(size_t)(s->ny / 2) * s->nx + x]);
    return nk[(size_t)((s->ny - 1) / 2) * s->nx + x];
}

static double first_down_crossing(const double* v, int xs, int nx, double level) {
    for (int x = xs; x + 1 < nx; ++x)
        if (v[x] >= level && v[x + 1] < level)
            return x + (v[x] - level) / (v[x] - v[x + 1]);
    return NAN;
}

void orc_observe(orc_t* s, orc_obs* out) {
    compute_density(s);
    memset(out, 0, sizeof *out);
    out->t = s->t;
    int bad = 0;
    for (int k = 0; k < 2; ++k) {
        double m = 0.0;
        for (int y = 0; y < s->ny; ++y)
            for (int x = 0; x < s->nx; ++x) {
                if (is_solid(s, x, y)) continue;
                double v = s->n[NIDX(s, k, y, x)];
                if (!isfinite(v) || v < -1e-3) bad = 1;
                m += v;
            }
        out->mass[k] = m;
    }
    int xs = s->x0 / 2;
    double* phi = (double*)malloc(sizeof(double) * s->nx);
    for (int x = 0; x < s->nx; ++x) phi[x] = centre_value(s, 0, x) - centre_value(s, 1, x);
    out->z = first_down_crossing(phi, xs, s->nx, 0.0) - s->x0;
    double level = centre_value(s, 0, xs) / 3.0;
    const double* nA = s->n;
    out->precursor_lo = first_down_crossing(nA + (size_t)1 * s->nx, xs, s->nx, level) - s->x0;
    out->precursor_hi = first_down_crossing(nA + (size_t)(s->ny - 2) * s->nx, xs, s->nx, level) - s->x0;
    out->precursor = 0.5 * (out->precursor_lo + out->precursor_hi);
    out->flags = (phi[xs] < 0.0 ? 1 : 0) | (bad ? 2 : 0);
    free(phi);
}
