/*
 * FP64 CPU oracle of the binary Shan-Chen lattice Boltzmann model of
 * S. Chibbaro, "Capillary filling with pseudo-potential binary Lattice-Boltzmann model".
 *
 * TEST INFRASTRUCTURE ONLY.  This code is the plain, slow reference the HIP library is
 * checked against.  Only the tests, the smoke check and the CPU-baseline leg of the bench
 * may load it; the product path never does.  It shares no code with the HIP library.
 *
 * Every step follows Sec. 2 of the paper in the paper's order: densities and momenta,
 * the bulk pseudo-potential force (eq. forcing) and the wall force (eq. forcingw), the
 * common velocity U, the shifted equilibrium velocity, the equilibrium (eqs. feq1-feq3),
 * BGK relaxation (eq. lbe) and streaming with bounce-back at solid nodes (Sec. 3).
 */
#ifndef SCF_ORACLE_H
#define SCF_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc orc_t;

typedef struct {
    int64_t t;
    double mass[2];        /* sum of n_k over fluid nodes */
    double z;              /* centreline interface position relative to x0, NaN if none */
    double precursor;      /* mean of the two wall-row precursor positions, NaN if either is absent */
    double precursor_lo;   /* row y = 1 */
    double precursor_hi;   /* row y = ny-2 */
    int32_t flags;         /* bit0: liquid reservoir exhausted; bit1: non-finite or negative density */
} orc_obs;

/* Geometry: nx by ny, solid rows y=0, ny-1 for x in [x0, x1).  periodic_x = 0 clamps x at
 * the box edges instead of wrapping (used only to run a window of a larger box). */
orc_t* orc_create(int nx, int ny, int x0, int x1, int periodic_x,
                  double G, const double gw[2], const double tau[2],
                  const double alpha[2], const double mass[2]);
void orc_destroy(orc_t*);
/* Optional solid mask, ny*nx row-major, non-zero = solid; it replaces the wall rows of
 * orc_create (x0, x1 then only place the observables).  Copied.  NULL restores the rows.
 * Call before orc_init. */
void orc_set_mask(orc_t*, const unsigned char* mask);
void orc_set_threads(int nthreads);
int  orc_threads(void);

/* f^k_i = f^{k(eq)}_i(n_k, u = 0); rho arrays are ny*nx row-major (x fastest). */
void orc_init(orc_t*, const double* rhoA, const double* rhoB);
void orc_collide(orc_t*);          /* post-collision values into the scratch array */
void orc_stream(orc_t*);           /* streaming with bounce-back, advances t */
void orc_step(orc_t*, int64_t nsteps);
int64_t orc_time(const orc_t*);

/* Macroscopic fields at the current state, each ny*nx per component (solid nodes 0):
 * n[2], j[2][2] (x then y), F[2][2] (bulk + wall), U[2] (x, y), ueq[2][2]. Any may be NULL. */
void orc_macro(orc_t*, double* n, double* j, double* F, double* U, double* ueq);
void orc_get_f(const orc_t*, double* f);            /* f[k][i][y][x] */
void orc_set_f(orc_t*, const double* f);
void orc_density(orc_t*, double* nA, double* nB);
void orc_observe(orc_t*, orc_obs* out);

/* Equilibrium of eqs. feq1-feq3 for one node. */
void orc_feq(double n, double ux, double uy, double alpha, double out[9]);

/* Three-dimensional D3Q19 counterpart (scf3d_oracle.c): box nx*ny*nz periodic in x, y, z;
 * solid nodes for x in [x0, x1) on the planes y = 0, ny-1 (walls_y) and z = 0, nz-1 (walls_z).
 * Arrays are nz*ny*nx (x fastest); populations f[k][i][z][y][x], i = 0..18 in the order of
 * the C arrays CX3, CY3, CZ3 of scf3d_oracle.c. */
typedef struct orc3 orc3_t;
orc3_t* orc3_create(int nx, int ny, int nz, int x0, int x1, int walls_y, int walls_z, double G,
                    const double gw[2], const double tau[2], const double mass[2]);
void orc3_destroy(orc3_t*);
void orc3_init(orc3_t*, const double* rhoA, const double* rhoB);
void orc3_step(orc3_t*, int64_t nsteps);
int64_t orc3_time(const orc3_t*);
void orc3_density(orc3_t*, double* nA, double* nB);
void orc3_get_f(const orc3_t*, double* f);
void orc3_set_f(orc3_t*, const double* f);
void orc3_observe(orc3_t*, double mass[2], double* z_front);
void orc3_feq(double n, double ux, double uy, double uz, double out[19]);

#ifdef __cplusplus
}
#endif
#endif
