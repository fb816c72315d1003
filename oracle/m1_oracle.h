/*
 * m1_oracle.h -- FP64 CPU reference ("oracle") for one explicit M1
 * radiative-transfer step fused with hydrogen photo-chemistry.
 *
 * TEST INFRASTRUCTURE ONLY.  This code is the independent checker of the
 * GPU library: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark may load it.  It shares no source, header, table or helper
 * with the HIP path, and the HIP path never calls it.
 *
 * Method (Aubert & Teyssier 2010, "Reionization simulations powered by
 * GPUs I"):
 *   - Sec. 2.2: two-moment equations for the photon number density N and
 *     the photon flux F in one frequency group, closed by P = D N with the
 *     M1 Eddington tensor D(chi, n); explicit time integration under the
 *     light-crossing (CFL) condition; Lax-Friedrichs intercell fluxes;
 *     hydrogen chemistry and cooling sub-cycled inside a transport step;
 *     the gray constants sigma_n, sigma_e and e_gamma.
 *   - Sec. 2.3: point sources projected on the grid by nearest grid point,
 *     each cell one source.
 *   - Appendix A: the conservative explicit finite-difference update from
 *     time p to p+1 (the 1-D form and its unsplit multi-dimensional sum),
 *     then the per-cell operator Phi that applies chemistry, temperature and
 *     absorption to the transported state.
 *
 * Readings where the paper is silent or garbled:
 *   closure chi(f) = Levermore form; D = (1-chi)/2 I + (3chi-1)/2 n(x)n
 *   (the printed coefficients are swapped); LF dissipation speed c; case-B
 *   rates of Hui & Gnedin (1997) and Cen (1992); photon-conserving implicit
 *   photoionisation, Anninos-style creation/destruction update for
 *   recombination, semi-implicit energy update.
 *
 * Layout: every field is FP64, row-major with x fastest.  N, Fx, Fy, Fz are
 * PADDED arrays of (nz+2)(ny+2)(nx+2) with a one-cell ghost layer; xHI, T,
 * nH and S are UNPADDED arrays of nz*ny*nx.
 */
#ifndef M1_ORACLE_H
#define M1_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* boundary condition per face (-x,+x,-y,+y,-z,+z) */
#define ORC_BC_PERIODIC 0
#define ORC_BC_OUTFLOW 1 /* zero-gradient copy                              */
#define ORC_BC_REFLECT 2 /* copy with the face-normal flux negated          */
#define ORC_BC_GIVEN 3   /* ghost values supplied by the caller (sub-block) */

/* chemistry modes */
#define ORC_CHEM_FULL 0       /* photoionisation + recombination + energy    */
#define ORC_CHEM_ISOTHERMAL 1 /* as FULL but T held fixed                    */
#define ORC_CHEM_OFF 2        /* transport and sources only                  */
#define ORC_CHEM_FROZEN 3     /* absorption by a fixed neutral density only  */

/* intercell flux (Sec. 2.2 names both; the paper's runs use LF) */
#define ORC_FLUX_LF 0  /* Lax-Friedrichs (Rusanov), dissipation speed c          */
#define ORC_FLUX_HLL 1 /* HLL with the extreme eigenvalues of the flux Jacobian */

/* sub-cycle modes */
#define ORC_SUB_FIXED 0
#define ORC_SUB_ADAPTIVE 1

/* Subgrid clumping (Sec. 3.2.1, "Clumping factors"): the cell-averaged
 * chemistry equation carries a recombination clumping factor C_R and a
 * photon/neutral cross clumping factor C_I, fitted in the paper as power
 * laws of the cell density.  Here
 *   C_R(nH) = max(1, cr_norm * nH^cr_exp)   (a ratio <y^2>/<y>^2 >= 1),
 *   C_I(nH) = ci_norm * nH^ci_exp,          nH in cm^-3.
 * C_I multiplies the photoionisation (and so the photon absorption) rate;
 * C_R multiplies every term in ne * nHII: case-B recombination, its
 * cooling and bremsstrahlung.  clump = 0 means C_R = C_I = 1.          */
typedef struct {
    int32_t nx, ny, nz;
    int32_t bc[6];
    int32_t chem;
    int32_t sub;
    int32_t clump;    /* 0 off, 1 power-law clumping factors    */
    int32_t flux;     /* ORC_FLUX_LF or ORC_FLUX_HLL            */
    double dx;        /* cell size [cm]                         */
    double c;         /* speed of light [cm/s]                  */
    double sigma_n;   /* number-averaged cross-section [cm^2]   */
    double sigma_e;   /* energy-averaged cross-section [cm^2]   */
    double egamma_eV; /* mean ionising photon energy [eV]       */
    double T_floor;   /* temperature floor [K]                  */
    double sub_eps;   /* adaptive sub-cycle fraction            */
    double cr_norm, cr_exp, ci_norm, ci_exp; /* clumping laws   */
    double hubble;    /* expansion rate H = (da/dt)/a [1/s], >= 0 (0: none)
                       * -- see orc_step_flux                    */
} orc_params;

/* tallies of one step, in photons (dt and cell volume folded in):
 * [0] absorbed, [1] escaped through outflow faces, [2] added by the N >= 0
 * floor, [3] chemistry sub-cycles executed (summed over cells), [4] removed
 * by the expansion's dilution.                                           */
#define ORC_NTALLY 5

double orc_chi(double f);
void orc_eddington(double N, double Fx, double Fy, double Fz, double c,
                   double P[6]); /* xx, yy, zz, xy, xz, yz */
void orc_rates(double T, double r[6]);
double orc_heat_per_ionisation_erg(const orc_params *p);
void orc_clumping(const orc_params *p, double nH, double *C_R, double *C_I);
/* orc_rates for n temperatures: r[6 i + m] = rate m at T[i]. */
void orc_rates_n(int64_t n, const double *T, double *r);
/* The adaptive sub-cycle time scale of a cell (the time over which the
 * chemistry changes xHI or the internal energy by their own size, from the
 * gross rates at the given state); INFINITY where nothing changes. */
double orc_chem_timescale(const orc_params *p, double nH, double N, double xHI,
                          double T);

void orc_chem_cell(const orc_params *p, double dt, int32_t nsub, double nH,
                   double *N, double *Fx, double *Fy, double *Fz, double *xHI,
                   double *T, double *absorbed, int32_t *ncycles);

void orc_sources_to_field(const orc_params *p, int64_t n, const int32_t *ijk,
                          const double *ndot, double *S);

void orc_fill_ghosts(const orc_params *p, double *N, double *Fx, double *Fy,
                     double *Fz);

int32_t orc_step(const orc_params *p, double dt, int32_t nsub, double *N,
                 double *Fx, double *Fy, double *Fz, double *xHI, double *T,
                 const double *nH, const double *S, double *tally);

/* One step as orc_step, with HLL face fluxes when p->flux == ORC_FLUX_HLL:
 * lam holds, for every cell of the PADDED grid (ghosts included, filled
 * from the boundary conditions before the call), the smallest and largest
 * eigenvalue of the flux Jacobian along x, y, z in units of c: 6 doubles
 * per cell (min x, max x, min y, max y, min z, max z). */
int32_t orc_step_flux(const orc_params *p, double dt, int32_t nsub, double *N,
                      double *Fx, double *Fy, double *Fz, double *xHI, double *T,
                      const double *nH, const double *S, const double *lam,
                      double *tally);
int32_t orc_run(const orc_params *p, double dt, int32_t nsub, int64_t nsteps,
                double *N, double *Fx, double *Fy, double *Fz, double *xHI,
                double *T, const double *nH, const double *S, double *tally);

#ifdef __cplusplus
}
#endif
#endif
