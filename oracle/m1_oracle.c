/*
 * m1_oracle.c -- FP64 CPU reference of the explicit M1 transport step and
 * the per-cell hydrogen chemistry operator.  TEST INFRASTRUCTURE ONLY (see
 * m1_oracle.h): plain loops, every quantity from its definition, no tiling,
 * no fusion beyond what the method itself states.  The adaptive sub-cycle
 * time scale is a reading (the paper states no rule), pinned by closed
 * forms of its consequences (marked where it is defined).  OpenMP only splits the
 * independent per-cell loops; every tally is summed per z-plane and then
 * over planes in a fixed order, so results do not depend on thread count.
 */
#include "m1_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* physical constants (CGS) */
static const double KB = 1.380649e-16;     /* Boltzmann [erg/K]          */
static const double EV = 1.602176634e-12;  /* electron-volt [erg]        */
static const double E_ION_EV = 13.6;       /* H ionisation threshold     */
static const double XHI_MIN = 1e-12;       /* neutral-fraction floor     */

/* padded index of interior cell (i, j, k), 0-based interior coordinates */
#define PIDX(p, i, j, k)                                                     \
    (((size_t)((k) + 1) * (size_t)((p)->ny + 2) + (size_t)((j) + 1)) *       \
         (size_t)((p)->nx + 2) +                                             \
     (size_t)((i) + 1))
/* unpadded index */
#define UIDX(p, i, j, k)                                                     \
    (((size_t)(k) * (size_t)(p)->ny + (size_t)(j)) * (size_t)(p)->nx +       \
     (size_t)(i))

/* ------------------------------------------------------------------------
 * M1 closure.  Sec. 2.2: chi depends only on the reduced flux f = |F|/(cN)
 * and runs from 1/3 (diffusion) to 1 (free streaming).  The paper defers the
 * formula to its method paper; we take the Levermore (1984) form used by the
 * M1 model it cites (Gonzalez et al. 2007).
 * --------------------------------------------------------------------- */
double orc_chi(double f)
{
    return (3.0 + 4.0 * f * f) / (5.0 + 2.0 * sqrt(4.0 - 3.0 * f * f));
}

/* Sec. 2.2: P = D N with D = (1-chi)/2 I + (3chi-1)/2 n(x)n, n = F/|F|.
 * (The printed equation swaps the two coefficients; that form has trace
 * 4chi-1 and gives n(x)n/3 at f = 0, so the standard M1 tensor is used.)
 * Output order: xx, yy, zz, xy, xz, yz. */
void orc_eddington(double N, double Fx, double Fy, double Fz, double c,
                   double P[6])
{
    for (int m = 0; m < 6; ++m) P[m] = 0.0;
    if (!(N > 0.0)) return;
    double Fn = sqrt(Fx * Fx + Fy * Fy + Fz * Fz);
    double f = Fn / (c * N);
    if (f > 1.0) f = 1.0;
    double chi = orc_chi(f);
    double iso = 0.5 * (1.0 - chi);
    double dir = 0.5 * (3.0 * chi - 1.0);
    double n[3] = {0.0, 0.0, 0.0};
    if (Fn > 0.0) {
        n[0] = Fx / Fn;
        n[1] = Fy / Fn;
        n[2] = Fz / Fn;
    }
    P[0] = N * (iso + dir * n[0] * n[0]);
    P[1] = N * (iso + dir * n[1] * n[1]);
    P[2] = N * (iso + dir * n[2] * n[2]);
    P[3] = N * dir * n[0] * n[1];
    P[4] = N * dir * n[0] * n[2];
    P[5] = N * dir * n[1] * n[2];
}

/* component (k, d) of the symmetric pressure tensor stored as above */
static double pcomp(const double P[6], int k, int d)
{
    static const int map[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
    return P[map[k][d]];
}

/* ------------------------------------------------------------------------
 * Hydrogen rate coefficients (Sec. 2.2 names only "hydrogen with the
 * associated cooling processes"; the set below is the reading used here).
 *   r[0] alpha_B  case-B recombination          [cm^3/s]  Hui & Gnedin 1997
 *   r[1] beta     collisional ionisation        [cm^3/s]  Cen 1992
 *   r[2] case-B recombination cooling           [erg cm^3/s] Hui & Gnedin
 *   r[3] collisional excitation cooling (HI)    [erg cm^3/s] Cen 1992
 *   r[4] collisional ionisation cooling = 13.6 eV * beta
 *   r[5] free-free (bremsstrahlung) cooling     [erg cm^3/s] Cen 1992
 * Pinned: alpha_B against a published table; r[1]..r[5] against physics
 * that does not come from these fits (thresholds at the ionisation and
 * Lyman-alpha energies, 13.6 eV per collisional ionisation, an independent
 * ionisation-rate fit, the mean energy per case-B recombination, the
 * free-free Gaunt factor and the excitation collision strength implied by
 * textbook prefactors).  The paper gives no rates, so the set itself is a
 * reading, not a parity claim against the paper.
 * --------------------------------------------------------------------- */
void orc_rates(double T, double r[6])
{
    double lam = 2.0 * 157807.0 / T;
    r[0] = 2.753e-14 * pow(lam, 1.5) /
           pow(1.0 + pow(lam / 2.740, 0.407), 2.242);
    double damp = 1.0 + sqrt(T / 1e5);
    r[1] = 5.85e-11 * sqrt(T) * exp(-157809.1 / T) / damp;
    r[2] = 3.435e-30 * T * pow(lam, 1.970) /
           pow(1.0 + pow(lam / 2.250, 0.376), 3.720);
    r[3] = 7.5e-19 * exp(-118348.0 / T) / damp;
    r[4] = E_ION_EV * EV * r[1];
    double lt = 5.5 - log10(T);
    double gff = 1.1 + 0.34 * exp(-lt * lt / 3.0);
    r[5] = 1.42e-27 * gff * sqrt(T);
}

void orc_rates_n(int64_t n, const double *T, double *r)
{
    for (int64_t i = 0; i < n; ++i) orc_rates(T[i], r + 6 * i);
}

/* Sec. 2.2 gray constants: energy deposited per photoionisation is the
 * mean absorbed photon energy sigma_e e / sigma_n minus the 13.6 eV that
 * the ionisation itself consumes. */
double orc_heat_per_ionisation_erg(const orc_params *p)
{
    return (p->sigma_e * p->egamma_eV / p->sigma_n - E_ION_EV) * EV;
}

/* Clumping factors of a cell of density nH (see orc_params). */
void orc_clumping(const orc_params *p, double nH, double *C_R, double *C_I)
{
    if (!p->clump) {
        *C_R = 1.0;
        *C_I = 1.0;
        return;
    }
    *C_R = fmax(1.0, p->cr_norm * pow(nH, p->cr_exp));
    *C_I = p->ci_norm * pow(nH, p->ci_exp);
}

/* Net cooling rate Lambda [erg cm^-3 s^-1] for electron density ne = nHII
 * (pure hydrogen) and neutral density nHI; the ne * nHII terms carry the
 * recombination clumping factor C_R. */
static double cooling(const double r[6], double nHII, double nHI, double C_R)
{
    double ne = nHII;
    return C_R * ne * nHII * (r[2] + r[5]) + ne * nHI * (r[3] + r[4]);
}

/* Adaptive sub-cycle time scale: the shorter of the neutral-fraction and
 * internal-energy times, each against the GROSS rate of change (creation
 * plus destruction, heating plus cooling).  Against the net rate the time
 * scale would be ill-conditioned near equilibrium, where the net rate is a
 * small difference of large terms.  The paper states no sub-cycling rule;
 * the tests pin this one by closed forms: the sub-cycle count of linear
 * recombination growth, ceil(ln(1 + alpha nH dt / xHI0) / ln(1 + eps)), and
 * at coronal equilibrium, where the net rate vanishes and the gross rate
 * sets the count. */
double orc_chem_timescale(const orc_params *p, double nH, double N,
                          double xHI, double T)
{
    double r[6], C_R, C_I;
    orc_rates(T, r);
    orc_clumping(p, nH, &C_R, &C_I);
    double x = 1.0 - xHI;
    double gamma = C_I * p->c * p->sigma_n * N;
    double gross_x = C_R * r[0] * nH * x * x + (gamma + r[1] * nH * x) * xHI;
    double u = 1.5 * KB * nH * (1.0 + x) * T;
    double gross_u = gamma * nH * xHI * orc_heat_per_ionisation_erg(p) +
                     cooling(r, nH * x, nH * xHI, C_R);
    double t = INFINITY;
    if (gross_x > 0.0) t = fmin(t, xHI / gross_x);
    if (p->chem == ORC_CHEM_FULL && gross_u > 0.0) t = fmin(t, u / gross_u);
    return t;
}

/* ------------------------------------------------------------------------
 * Per-cell operator Phi (Appendix A): chemistry, temperature and absorption
 * applied to the transported photon state, sub-cycled within the step
 * (Sec. 2.2).  One sub-cycle of length h:
 *   1. photoionisation, backward Euler on the coupled pair
 *      dN/dt = dnHI/dt = -c sigma_n nHI N (photon conserving); the
 *      absorbed density P solves a (nHI - P)(N - P) = P, a = c sigma_n h,
 *      with 0 <= P <= min(N, nHI).  F is attenuated by the same factor
 *      as N (kappa is the same in both moment equations, Sec. 2.2);
 *   2. recombination (case B, on the spot) and collisional ionisation in
 *      creation/destruction form after Anninos et al. (1997):
 *      xHI <- (xHI + alpha_B nH x^2 h) / (1 + beta nH x h);
 *   3. internal energy u = 3/2 kB nH (1 + x) T gains P * e_heat and is
 *      cooled semi-implicitly, u <- (u + H)/(1 + h Lambda/u), with the rates
 *      at the sub-cycle's starting temperature.
 * With subgrid clumping (Sec. 3.2.1) a becomes C_I a and the ne nHII terms
 * (alpha_B, recombination cooling, bremsstrahlung) are multiplied by C_R.
 * --------------------------------------------------------------------- */
void orc_chem_cell(const orc_params *p, double dt, int32_t nsub, double nH,
                   double *N, double *Fx, double *Fy, double *Fz, double *xHI,
                   double *T, double *absorbed, int32_t *ncycles)
{
    double eheat = orc_heat_per_ionisation_erg(p);
    double C_R, C_I;
    orc_clumping(p, nH, &C_R, &C_I);
    double remaining = dt;
    int32_t it = 0;
    *absorbed = 0.0;
    for (it = 0; it < nsub && remaining > 0.0; ++it) {
        double h;
        if (it == nsub - 1) {
            h = remaining;
        } else if (p->sub == ORC_SUB_ADAPTIVE) {
            double tc = orc_chem_timescale(p, nH, *N, *xHI, *T);
            h = fmin(remaining, p->sub_eps * tc);
        } else {
            h = dt / nsub;
        }
        remaining -= h;
        if (it == nsub - 1 || remaining < 0.0) remaining = 0.0;

        double a = C_I * p->c * p->sigma_n * h;
        double x0 = 1.0 - *xHI;
        double nHI = nH * (*xHI);

        /* step 1: photoionisation */
        double Pabs;
        if (p->chem == ORC_CHEM_FROZEN) {
            Pabs = a * nHI * (*N) / (1.0 + a * nHI);
        } else {
            double B = 1.0 + a * (nHI + *N);
            double C = a * nHI * (*N);
            Pabs = 2.0 * C / (B + sqrt(B * B - 4.0 * a * C));
        }
        double Nold = *N;
        *N = Nold - Pabs;
        if (*N < 0.0) *N = 0.0;
        double scale = (Nold > 0.0) ? (*N / Nold) : 0.0;
        *Fx *= scale;
        *Fy *= scale;
        *Fz *= scale;
        *absorbed += Pabs;
        if (p->chem == ORC_CHEM_FROZEN) continue;
        *xHI -= Pabs / nH;

        /* step 2: recombination and collisional ionisation */
        double r[6];
        orc_rates(*T, r);
        double x = 1.0 - *xHI;
        double xn = (*xHI + C_R * r[0] * nH * x * x * h) / (1.0 + r[1] * nH * x * h);
        if (xn < XHI_MIN) xn = XHI_MIN;
        if (xn > 1.0) xn = 1.0;
        *xHI = xn;

        /* step 3: energy */
        if (p->chem == ORC_CHEM_FULL) {
            double x1 = 1.0 - xn;
            double u = 1.5 * KB * nH * (1.0 + x0) * (*T);
            double H = Pabs * eheat;
            double lam = cooling(r, nH * x1, nH * xn, C_R);
            u = (u + H) / (1.0 + h * lam / u);
            double Tn = u / (1.5 * KB * nH * (1.0 + x1));
            *T = (Tn > p->T_floor) ? Tn : p->T_floor;
        }
    }
    *ncycles = it;
}

/* Sec. 2.3: nearest-grid-point projection, every cell one source; emission
 * rate density S = Ndot / dx^3, duplicate cells summed. */
void orc_sources_to_field(const orc_params *p, int64_t n, const int32_t *ijk,
                          const double *ndot, double *S)
{
    double vol = p->dx * p->dx * p->dx;
    for (int64_t s = 0; s < n; ++s) {
        int i = ijk[3 * s], j = ijk[3 * s + 1], k = ijk[3 * s + 2];
        S[UIDX(p, i, j, k)] += ndot[s] / vol;
    }
}

/* ------------------------------------------------------------------------
 * Ghost layer from the boundary conditions (the paper pads its grids with
 * ghost layers, Appendix A; their content is not stated).
 * --------------------------------------------------------------------- */
static void ghost_copy(double *const U[4], size_t dst, size_t src, int bc,
                       int normal)
{
    if (bc == ORC_BC_GIVEN) return;
    for (int m = 0; m < 4; ++m) U[m][dst] = U[m][src];
    if (bc == ORC_BC_REFLECT) U[1 + normal][dst] = -U[1 + normal][dst];
}

void orc_fill_ghosts(const orc_params *p, double *N, double *Fx, double *Fy,
                     double *Fz)
{
    double *const U[4] = {N, Fx, Fy, Fz};
    int nx = p->nx, ny = p->ny, nz = p->nz;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j) {
            int lo = p->bc[0] == ORC_BC_PERIODIC ? nx - 1 : 0;
            int hi = p->bc[1] == ORC_BC_PERIODIC ? 0 : nx - 1;
            ghost_copy(U, PIDX(p, -1, j, k), PIDX(p, lo, j, k), p->bc[0], 0);
            ghost_copy(U, PIDX(p, nx, j, k), PIDX(p, hi, j, k), p->bc[1], 0);
        }
    for (int k = 0; k < nz; ++k)
        for (int i = 0; i < nx; ++i) {
            int lo = p->bc[2] == ORC_BC_PERIODIC ? ny - 1 : 0;
            int hi = p->bc[3] == ORC_BC_PERIODIC ? 0 : ny - 1;
            ghost_copy(U, PIDX(p, i, -1, k), PIDX(p, i, lo, k), p->bc[2], 1);
            ghost_copy(U, PIDX(p, i, ny, k), PIDX(p, i, hi, k), p->bc[3], 1);
        }
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            int lo = p->bc[4] == ORC_BC_PERIODIC ? nz - 1 : 0;
            int hi = p->bc[5] == ORC_BC_PERIODIC ? 0 : nz - 1;
            ghost_copy(U, PIDX(p, i, j, -1), PIDX(p, i, j, lo), p->bc[4], 2);
            ghost_copy(U, PIDX(p, i, j, nz), PIDX(p, i, j, hi), p->bc[5], 2);
        }
}

/* Lax-Friedrichs (Rusanov) intercell flux across a face normal to d between
 * the left state (UL, PL) and the right state (UR, PR), Sec. 2.2 and
 * Appendix A; dissipation speed c.  U = (N, Fx, Fy, Fz); the physical flux
 * of N along d is F_d and that of F_k is c^2 P_kd (moment equations). */
static void lf_flux(int d, const double UL[4], const double PL[6],
                    const double UR[4], const double PR[6], double c,
                    double G[4])
{
    G[0] = 0.5 * (UL[1 + d] + UR[1 + d]) - 0.5 * c * (UR[0] - UL[0]);
    for (int k = 0; k < 3; ++k)
        G[1 + k] = 0.5 * c * c * (pcomp(PL, k, d) + pcomp(PR, k, d)) -
                   0.5 * c * (UR[1 + k] - UL[1 + k]);
}

/* HLL (Sec. 2.2 names it beside LF): with the signal speeds
 * a+ = c max(0, lmax_L, lmax_R) and a- = c min(0, lmin_L, lmin_R),
 *   G = (a+ G(U_L) - a- G(U_R) + a+ a- (U_R - U_L)) / (a+ - a-). */
static void hll_flux(int d, const double UL[4], const double PL[6], const double lL[2],
                     const double UR[4], const double PR[6], const double lR[2],
                     double c, double G[4])
{
    double GL[4], GR[4];
    GL[0] = UL[1 + d];
    GR[0] = UR[1 + d];
    for (int k = 0; k < 3; ++k) {
        GL[1 + k] = c * c * pcomp(PL, k, d);
        GR[1 + k] = c * c * pcomp(PR, k, d);
    }
    double ap = c * fmax(0.0, fmax(lL[1], lR[1]));
    double am = c * fmin(0.0, fmin(lL[0], lR[0]));
    if (!(ap - am > 0.0)) {
        for (int m = 0; m < 4; ++m) G[m] = 0.5 * (GL[m] + GR[m]);
        return;
    }
    for (int m = 0; m < 4; ++m)
        G[m] = (ap * GL[m] - am * GR[m] + ap * am * (UR[m] - UL[m])) / (ap - am);
}

static int check_params(const orc_params *p)
{
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return -1;
    for (int f = 0; f < 6; ++f)
        if (p->bc[f] < 0 || p->bc[f] > ORC_BC_GIVEN) return -1;
    for (int d = 0; d < 3; ++d)
        if ((p->bc[2 * d] == ORC_BC_PERIODIC) !=
            (p->bc[2 * d + 1] == ORC_BC_PERIODIC))
            return -1;
    if (p->chem < 0 || p->chem > ORC_CHEM_FROZEN) return -1;
    if (p->sub != ORC_SUB_FIXED && p->sub != ORC_SUB_ADAPTIVE) return -1;
    if (!(p->dx > 0.0) || !(p->c > 0.0)) return -1;
    if (p->flux != ORC_FLUX_LF && p->flux != ORC_FLUX_HLL) return -1;
    if (!(p->hubble >= 0.0) || !isfinite(p->hubble)) return -1;
    return 0;
}

/* ------------------------------------------------------------------------
 * One radiative-transfer step (Appendix A): all face fluxes from the step-p
 * state, the unsplit update
 *     u~ = u - dt/dx * sum_d (G_{d,+1/2} - G_{d,-1/2}) + dt S   (S on N),
 * then Phi per cell.  Returns 0, or -1 on invalid parameters.
 *
 * Expansion (p->hubble = H > 0).  The moment equations of Sec. 2.2 carry no
 * expansion terms, while the runs cover some 800 Myr of cosmic time on
 * comoving boxes (Sec. 2.1-2.3).  Reading: in proper units, a homogeneous
 * expansion at rate H dilutes the photon number density and the photon
 * number flux alike, dN/dt = -3 H N and dF/dt = -3 H F (each photon keeps
 * its direction and speed, so the reduced flux |F|/(cN), hence the M1
 * closure, is unchanged; photons redshifting out of the single group are
 * not followed), and cools the gas adiabatically, dT/dt = -2 H T for a
 * monatomic ideal gas (full chemistry only: the isothermal mode holds T by
 * definition, the frozen mode holds the gas).  The gas density is the
 * snapshot's, as given.  Operator split, with H constant over the step and
 * the two linear equations solved exactly: after the transport update and
 * its guards, N, F *= exp(-3 H dt) and T *= exp(-2 H dt), then Phi.
 * --------------------------------------------------------------------- */
int32_t orc_step(const orc_params *p, double dt, int32_t nsub, double *N,
                 double *Fx, double *Fy, double *Fz, double *xHI, double *T,
                 const double *nH, const double *S, double *tally)
{
    return orc_step_flux(p, dt, nsub, N, Fx, Fy, Fz, xHI, T, nH, S, NULL, tally);
}

int32_t orc_step_flux(const orc_params *p, double dt, int32_t nsub, double *N,
                      double *Fx, double *Fy, double *Fz, double *xHI, double *T,
                      const double *nH, const double *S, const double *lam,
                      double *tally)
{
    if (check_params(p) != 0 || nsub < 1 || !(dt > 0.0)) return -1;
    if (p->flux == ORC_FLUX_HLL && !lam) return -1;
    const int nx = p->nx, ny = p->ny, nz = p->nz;
    const size_t npad = (size_t)(nx + 2) * (ny + 2) * (nz + 2);
    const double c = p->c, vol = p->dx * p->dx * p->dx;
    const double k1 = dt / p->dx;

    orc_fill_ghosts(p, N, Fx, Fy, Fz);

    /* closure everywhere, ghosts included */
    double *P = (double *)calloc(6 * npad, sizeof(double));
    double *Un = (double *)malloc(4 * npad * sizeof(double));
    double *plane = (double *)calloc((size_t)nz * ORC_NTALLY, sizeof(double));
    if (!P || !Un || !plane) {
        free(P);
        free(Un);
        free(plane);
        return -2;
    }
#pragma omp parallel for schedule(static)
    for (long long q = 0; q < (long long)npad; ++q)
        orc_eddington(N[q], Fx[q], Fy[q], Fz[q], c, P + 6 * q);

    const double *U[4] = {N, Fx, Fy, Fz};
    const size_t stride[3] = {1, (size_t)(nx + 2),
                              (size_t)(nx + 2) * (size_t)(ny + 2)};
    const int ext[3] = {nx, ny, nz};

#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k) {
        double *tl = plane + (size_t)k * ORC_NTALLY;
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const int ijk[3] = {i, j, k};
                size_t q = PIDX(p, i, j, k);
                double Uc[4], div[4] = {0, 0, 0, 0};
                for (int m = 0; m < 4; ++m) Uc[m] = U[m][q];
                for (int d = 0; d < 3; ++d) {
                    size_t qm = q - stride[d], qp = q + stride[d];
                    double Um[4], Up[4], Gm[4], Gp[4];
                    for (int m = 0; m < 4; ++m) {
                        Um[m] = U[m][qm];
                        Up[m] = U[m][qp];
                    }
                    if (p->flux == ORC_FLUX_HLL) {
                        hll_flux(d, Um, P + 6 * qm, lam + 6 * qm + 2 * d, Uc, P + 6 * q,
                                 lam + 6 * q + 2 * d, c, Gm);
                        hll_flux(d, Uc, P + 6 * q, lam + 6 * q + 2 * d, Up, P + 6 * qp,
                                 lam + 6 * qp + 2 * d, c, Gp);
                    } else {
                        lf_flux(d, Um, P + 6 * qm, Uc, P + 6 * q, c, Gm);
                        lf_flux(d, Uc, P + 6 * q, Up, P + 6 * qp, c, Gp);
                    }
                    for (int m = 0; m < 4; ++m) div[m] += Gp[m] - Gm[m];
                    /* photons leaving through outflow faces */
                    if (ijk[d] == 0 && p->bc[2 * d] == ORC_BC_OUTFLOW)
                        tl[1] += -Gm[0] * dt * p->dx * p->dx;
                    if (ijk[d] == ext[d] - 1 &&
                        p->bc[2 * d + 1] == ORC_BC_OUTFLOW)
                        tl[1] += Gp[0] * dt * p->dx * p->dx;
                }
                double Nt = Uc[0] - k1 * div[0];
                if (S) Nt += dt * S[UIDX(p, i, j, k)];
                double Ft[3];
                for (int m = 0; m < 3; ++m) Ft[m] = Uc[1 + m] - k1 * div[1 + m];

                /* guards: N >= 0 and |F| <= c N */
                if (Nt < 0.0) {
                    tl[2] += -Nt * vol;
                    Nt = 0.0;
                }
                double Fn = sqrt(Ft[0] * Ft[0] + Ft[1] * Ft[1] + Ft[2] * Ft[2]);
                if (Fn > c * Nt) {
                    double s = (Fn > 0.0) ? c * Nt / Fn : 0.0;
                    for (int m = 0; m < 3; ++m) Ft[m] *= s;
                }
                /* expansion: dilution over the step */
                if (p->hubble > 0.0) {
                    const double e3 = exp(-3.0 * p->hubble * dt);
                    tl[4] += (1.0 - e3) * Nt * vol;
                    Nt *= e3;
                    for (int m = 0; m < 3; ++m) Ft[m] *= e3;
                }
                Un[0 * npad + q] = Nt;
                Un[1 * npad + q] = Ft[0];
                Un[2 * npad + q] = Ft[1];
                Un[3 * npad + q] = Ft[2];
            }
    }

    /* Phi: chemistry, temperature, absorption, per cell */
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k) {
        double *tl = plane + (size_t)k * ORC_NTALLY;
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t q = PIDX(p, i, j, k), u = UIDX(p, i, j, k);
                double Nn = Un[q], fx = Un[npad + q], fy = Un[2 * npad + q],
                       fz = Un[3 * npad + q];
                /* expansion: adiabatic cooling of the gas over the step */
                if (p->hubble > 0.0 && p->chem == ORC_CHEM_FULL)
                    T[u] *= exp(-2.0 * p->hubble * dt);
                if (p->chem != ORC_CHEM_OFF) {
                    double abs_ = 0.0;
                    int32_t nc = 0;
                    orc_chem_cell(p, dt, nsub, nH[u], &Nn, &fx, &fy, &fz,
                                  &xHI[u], &T[u], &abs_, &nc);
                    tl[0] += abs_ * vol;
                    tl[3] += nc;
                }
                N[q] = Nn;
                Fx[q] = fx;
                Fy[q] = fy;
                Fz[q] = fz;
            }
    }

    for (int m = 0; m < ORC_NTALLY; ++m) tally[m] = 0.0;
    for (int k = 0; k < nz; ++k)
        for (int m = 0; m < ORC_NTALLY; ++m)
            tally[m] += plane[(size_t)k * ORC_NTALLY + m];
    free(P);
    free(Un);
    free(plane);
    return 0;
}

/* nsteps consecutive steps of orc_step; tallies summed over the steps */
int32_t orc_run(const orc_params *p, double dt, int32_t nsub, int64_t nsteps,
                double *N, double *Fx, double *Fy, double *Fz, double *xHI,
                double *T, const double *nH, const double *S, double *tally)
{
    double acc[ORC_NTALLY] = {0, 0, 0, 0, 0}, one[ORC_NTALLY];
    for (int64_t s = 0; s < nsteps; ++s) {
        int32_t rc = orc_step(p, dt, nsub, N, Fx, Fy, Fz, xHI, T, nH, S, one);
        if (rc != 0) return rc;
        for (int m = 0; m < ORC_NTALLY; ++m) acc[m] += one[m];
    }
    for (int m = 0; m < ORC_NTALLY; ++m) tally[m] = acc[m];
    return 0;
}
