/*
 * gb_oracle.c -- plain FP64 CPU oracle for the GB-OBC electrostatics and the
 * discrete-state Monte Carlo / E-REMD decisions of constant redox potential
 * MD (CEMD), coupled constant pH and redox MD (C(pH,E)MD) and redox potential
 * replica exchange (E-REMD), Cruzeiro, Amaral & Roitberg, arXiv:1803.09652.
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  It shares no code, header,
 * table or constant with the GPU library; neither includes the other.
 *
 * Everything is the plain definition: O(N^2) double loops over atom pairs in
 * FP64, no blocking, no fixed point, no series expansions.  Full rows are
 * computed per atom (each ordered pair visited from both ends), which lets
 * OpenMP split the outer loop with no reductions across threads.
 *
 * Model (the paper names the Onufriev-Bashford-Case GB model, section III.D/E,
 * but prints no formula; these are the published HCT/OBC/Still definitions):
 *   rt_i = rho_i - offset;  S_j = screen_j * rt_j
 *   H(r; rt, S)  = (1/4pi) * integral of |x|^-4 over the part of a ball of
 *                  radius S at distance r that lies outside the ball of radius
 *                  rt around the origin (closed form in or_hct)
 *   I_i = sum_{j!=i} H(r_ij; rt_i, S_j);  Psi_i = rt_i I_i
 *   theta_i = alpha Psi - beta Psi^2 + gamma Psi^3
 *   R_i = 1 / (1/rt_i - tanh(theta_i)/rho_i)
 *   f_ij = sqrt(r^2 + R_i R_j exp(-r^2/(4 R_i R_j))),  f_ii = R_i
 *   E_C  = k sum_{i<j} q_i q_j / (eps_in r_ij)
 *   E_GB = -(k / 2) sum_i sum_j q_i q_j d(f_ij) / f_ij,
 *   d(f) = 1/eps_in - exp(-kappa f)/eps_out   (salt: the Debye-Hueckel factor
 *          of Srinivasan et al., Theor. Chem. Acc. 101 (1999) 426; with
 *          kappa = 0, d = tau = 1/eps_in - 1/eps_out)
 * Units: Angstrom, elementary charge, kcal/mol, volt, kelvin.
 *
 * Monte Carlo (section II.A-B): Delta G of a proposed state is Eq. 8 (redox)
 * or Eq. 9 (protonation) in their multi-state form; Metropolis acceptance.
 * Replica exchange (section II.C): Eq. 14 and Eq. 15.
 * Cutoffs (optional; the paper's runs have none): rgbmax restricts the
 * descreening integral to the sphere of that radius around each atom
 * (or_hct_cut); cutoff drops the Coulomb and GB pair terms of pairs at or
 * beyond that distance (self terms stay).
 * Dynamics between attempts (section III.D: Langevin thermostat): the leapfrog
 * Langevin scheme of Loncharich, Brooks and Pastor (Biopolymers 32, 523,
 * 1992) on the electrostatic forces, plus an optional harmonic restraint of
 * every atom to reference coordinates standing in for the bonded and van der
 * Waals terms of a full force field.  Units: ps, amu, Angstrom/ps.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_KB 1.98720426e-3        /* kcal/(mol K): CODATA R / 4184 */
#define OR_FARADAY 23.0605478      /* kcal/(mol V): CODATA F / 4184 */
#define OR_LN10 2.302585092994045684
/* 1 kcal/mol per (amu Angstrom) in Angstrom/ps^2: 4184 J / 1e-3 kg, in A^2/ps^2 */
#define OR_ACC 418.4

typedef struct {
    double alpha, beta, gamma, offset, eps_in, eps_out, coulomb_k;
    double kappa;   /* inverse Debye length (1/A); 0: no salt */
    double rgbmax;  /* descreening cutoff (A); 0: none */
    double cutoff;  /* pair cutoff of the energy terms (A); 0: none */
} or_params;

double or_kb(void) { return OR_KB; }
double or_faraday(void) { return OR_FARADAY; }

/* ------------------------------------------------------------------------
 * HCT pair integral.  With U = r + S and L = max(rt, |r - S|):
 *   0                                                   if rt >= U
 *   1/2 [1/L - 1/U + r/4 (1/U^2 - 1/L^2) + ln(L/U)/(2r)
 *        + S^2/(4r) (1/L^2 - 1/U^2)]
 *   + (1/rt - 1/L)           if rt < S - r (the origin lies inside ball j:
 *                            the full shells between rt and S - r)
 * ------------------------------------------------------------------------ */
double or_hct(double r, double rt, double S)
{
    double U = r + S;
    if (rt >= U) return 0.0;
    double L = fabs(r - S);
    if (rt > L) L = rt;
    double a = 1.0 / L, b = 1.0 / U;
    double h = a - b + 0.25 * r * (b * b - a * a) + 0.5 / r * log(L / U)
             + 0.25 * S * S / r * (a * a - b * b);
    double H = 0.5 * h;
    if (rt < S - r) H += 1.0 / rt - a;
    return H;
}

/* Partial derivatives of or_hct: out[0] = dH/dr, out[1] = dH/drt, out[2] = dH/dS.
 * The bracket h(L, U, r, S) has dh/dU = 0 at U = r + S and dh/dL = 0 at
 * L = r - S; in the engulfed case (L = S - r) the L-dependence of h cancels
 * against the -1/L of the full-shell term.  So dH/dr and dH/dS are the explicit
 * partials of h/2 at fixed (L, U), and H depends on rt only where L = rt or in
 * the engulfed full-shell term. */
void or_hct_grad(double r, double rt, double S, double* out)
{
    out[0] = out[1] = out[2] = 0.0;
    double U = r + S;
    if (rt >= U) return;
    double L = fabs(r - S);
    int l_is_rt = 0;
    if (rt > L) { L = rt; l_is_rt = 1; }
    double a = 1.0 / L, b = 1.0 / U;
    /* dh/dr|_{L,U} = 1/4 (b^2 - a^2)(1 + S^2/r^2) - ln(L/U)/(2 r^2) */
    double dhdr = 0.25 * (b * b - a * a) * (1.0 + S * S / (r * r)) - log(L / U) / (2.0 * r * r);
    double dhdS = S / (2.0 * r) * (a * a - b * b);
    out[0] = 0.5 * dhdr;
    out[2] = 0.5 * dhdS;
    if (l_is_rt) {
        /* dh/dL = ((L - r)^2 - S^2) / (2 r L^3) */
        out[1] = 0.5 * ((L - r) * (L - r) - S * S) / (2.0 * r * L * L * L);
    } else if (rt < S - r) {
        out[1] = -1.0 / (rt * rt);
    }
}

/* H restricted to the sphere of radius c around atom i (the descreening
 * cutoff): the part of ball j that lies inside radius c and outside rt,
 *   H_c(r; rt, S) = H(r; rt, S) - H(r; c, S)   for c > rt,   0 for c <= rt,
 * since H(r; c, S) is the part of ball j outside radius c.  c <= 0: no cutoff. */
double or_hct_cut(double r, double rt, double S, double c)
{
    if (c <= 0.0) return or_hct(r, rt, S);
    if (c <= rt) return 0.0;
    return or_hct(r, rt, S) - or_hct(r, c, S);
}

/* Partials of or_hct_cut (dr, drt, dS); the c term does not depend on rt. */
void or_hct_cut_grad(double r, double rt, double S, double c, double* out)
{
    or_hct_grad(r, rt, S, out);
    if (c <= 0.0) return;
    if (c <= rt) { out[0] = out[1] = out[2] = 0.0; return; }
    double g[3];
    or_hct_grad(r, c, S, g);
    out[0] -= g[0];
    out[2] -= g[2];
}

/* 1 if the pair at distance r lies beyond the energy cutoff (its Coulomb and
 * GB pair terms are dropped; self terms never are). */
static inline int beyond(const or_params* p, double r)
{
    return p->cutoff > 0.0 && r >= p->cutoff;
}

static inline double dist(const double* x, const double* y, const double* z, int i, int j)
{
    double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
    return sqrt(dx * dx + dy * dy + dz * dz);
}

/* Born radii of one system.  Outputs (each [n], any may be NULL):
 * I (descreening sum), R (effective Born radius), T = tanh(theta),
 * dRdPsi = dR/dPsi. */
void or_radii(int n, const double* x, const double* y, const double* z,
              const double* rho, const double* screen, const or_params* p,
              double* I, double* R, double* T, double* dRdPsi)
{
    #pragma omp parallel for schedule(dynamic, 16)
    for (int i = 0; i < n; ++i) {
        double rt = rho[i] - p->offset;
        double sum = 0.0;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            double Sj = screen[j] * (rho[j] - p->offset);
            sum += or_hct_cut(dist(x, y, z, i, j), rt, Sj, p->rgbmax);
        }
        double psi = rt * sum;
        double th = p->alpha * psi - p->beta * psi * psi + p->gamma * psi * psi * psi;
        double t = tanh(th);
        double Ri = 1.0 / (1.0 / rt - t / rho[i]);
        if (I) I[i] = sum;
        if (R) R[i] = Ri;
        if (T) T[i] = t;
        if (dRdPsi)
            dRdPsi[i] = Ri * Ri * (1.0 - t * t)
                      * (p->alpha - 2.0 * p->beta * psi + 3.0 * p->gamma * psi * psi) / rho[i];
    }
}

/* Dielectric factor of one GB pair term (or self term, f = R_i):
 * d(f) = 1/eps_in - exp(-kappa f)/eps_out. */
static inline double gb_d(const or_params* p, double f)
{
    return 1.0 / p->eps_in - exp(-p->kappa * f) / p->eps_out;
}

/* Its slope factor: d/df [d(f)/f] = -gb_s(f) / f^2 with
 * gb_s(f) = d(f) - kappa f exp(-kappa f) / eps_out (= tau when kappa = 0). */
static inline double gb_s(const or_params* p, double f)
{
    return gb_d(p, f) - p->kappa * f * exp(-p->kappa * f) / p->eps_out;
}

/* Still's f_GB and its partials for i != j. */
static inline void fgb(double r, double Ri, double Rj, double* f, double* ex, double* D)
{
    double RR = Ri * Rj;
    *D = r * r / (4.0 * RR);
    *ex = exp(-*D);
    *f = sqrt(r * r + RR * *ex);
}

/* Energies (out_E[0] = E_C, out_E[1] = E_GB) at *given* Born radii R. */
void or_energy_fixedR(int n, const double* x, const double* y, const double* z,
                      const double* q, const double* R, const or_params* p, double* out_E)
{
    double k = p->coulomb_k;
    double ec = 0.0, eg = 0.0;
    #pragma omp parallel for schedule(dynamic, 16) reduction(+ : ec, eg)
    for (int i = 0; i < n; ++i) {
        double ci = 0.0, gi = 0.0;
        for (int j = 0; j < n; ++j) {
            if (j == i) { gi += q[i] * q[i] * gb_d(p, R[i]) / R[i]; continue; }
            double r = dist(x, y, z, i, j), f, ex, D;
            if (beyond(p, r)) continue;
            fgb(r, R[i], R[j], &f, &ex, &D);
            if (j > i) ci += q[i] * q[j] / (p->eps_in * r);
            gi += q[i] * q[j] * gb_d(p, f) / f;
        }
        ec += ci;
        eg += gi;
    }
    out_E[0] = k * ec;
    out_E[1] = -0.5 * k * eg;
}

/* Charge gradient phi_i = dE/dq_i at given Born radii (self term included). */
void or_phi_fixedR(int n, const double* x, const double* y, const double* z,
                   const double* q, const double* R, const or_params* p, double* phi)
{
    double k = p->coulomb_k;
    #pragma omp parallel for schedule(dynamic, 16)
    for (int i = 0; i < n; ++i) {
        double s = -k * gb_d(p, R[i]) * q[i] / R[i];
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            double r = dist(x, y, z, i, j), f, ex, D;
            if (beyond(p, r)) continue;
            fgb(r, R[i], R[j], &f, &ex, &D);
            s += k * q[j] / (p->eps_in * r) - k * gb_d(p, f) * q[j] / f;
        }
        phi[i] = s;
    }
}

/* Full evaluation of one system: radii, energies and all gradients.
 * out_E[2] = {E_C, E_GB};  F[3n] = -dE/dx (x-block, y-block, z-block);
 * phi[n] = dE/dq;  dEdrho[n] = dE/drho (intrinsic radius);  G[n] = dE/dR;
 * R[n] = Born radii.  Any output pointer except out_E may be NULL. */
void or_energy_forces(int n, const double* x, const double* y, const double* z,
                      const double* q, const double* rho, const double* screen,
                      const or_params* p, double* out_E, double* F, double* phi,
                      double* dEdrho, double* Gout, double* Rout)
{
    double k = p->coulomb_k;
    double* I = malloc(sizeof(double) * n);
    double* R = malloc(sizeof(double) * n);
    double* T = malloc(sizeof(double) * n);
    double* dRdPsi = malloc(sizeof(double) * n);
    double* G = malloc(sizeof(double) * n);
    double* B = malloc(sizeof(double) * n);
    or_radii(n, x, y, z, rho, screen, p, I, R, T, dRdPsi);
    or_energy_fixedR(n, x, y, z, q, R, p, out_E);

    /* explicit pair forces, G = dE/dR, phi = dE/dq */
    #pragma omp parallel for schedule(dynamic, 16)
    for (int i = 0; i < n; ++i) {
        double fx = 0, fy = 0, fz = 0;
        double g = 0.5 * k * gb_s(p, R[i]) * q[i] * q[i] / (R[i] * R[i]);
        double ph = -k * gb_d(p, R[i]) * q[i] / R[i];
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
            double r = sqrt(dx * dx + dy * dy + dz * dz), f, ex, D;
            if (beyond(p, r)) continue;
            fgb(r, R[i], R[j], &f, &ex, &D);
            double qq = q[i] * q[j];
            double dfdr = r / f * (1.0 - 0.25 * ex);
            double sf = gb_s(p, f);
            double dEdr = -k * qq / (p->eps_in * r * r) + k * sf * qq / (f * f) * dfdr;
            fx -= dEdr * dx / r;
            fy -= dEdr * dy / r;
            fz -= dEdr * dz / r;
            double dfdRi = R[j] * ex * (1.0 + D) / (2.0 * f);
            g += k * sf * qq / (f * f) * dfdRi;
            ph += k * q[j] / (p->eps_in * r) - k * gb_d(p, f) * q[j] / f;
        }
        if (F) { F[i] = fx; F[n + i] = fy; F[2 * n + i] = fz; }
        G[i] = g;
        if (phi) phi[i] = ph;
    }
    for (int i = 0; i < n; ++i) B[i] = G[i] * dRdPsi[i];

    /* Born-radius chain: force through Psi and dE/drho */
    #pragma omp parallel for schedule(dynamic, 16)
    for (int a = 0; a < n; ++a) {
        double rta = rho[a] - p->offset, Sa = screen[a] * rta;
        double fx = 0, fy = 0, fz = 0, drt_sum = 0, dS_sum = 0;
        for (int j = 0; j < n; ++j) {
            if (j == a) continue;
            double rtj = rho[j] - p->offset, Sj = screen[j] * rtj;
            double dx = x[a] - x[j], dy = y[a] - y[j], dz = z[a] - z[j];
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            double gaj[3], gja[3];
            or_hct_cut_grad(r, rta, Sj, p->rgbmax, gaj);   /* H(r_aj; rt_a, S_j): in Psi_a */
            or_hct_cut_grad(r, rtj, Sa, p->rgbmax, gja);   /* H(r_ja; rt_j, S_a): in Psi_j */
            double dEdr = B[a] * rta * gaj[0] + B[j] * rtj * gja[0];
            fx -= dEdr * dx / r;
            fy -= dEdr * dy / r;
            fz -= dEdr * dz / r;
            drt_sum += gaj[1];
            dS_sum += B[j] * rtj * gja[2];
        }
        if (F) { F[a] += fx; F[n + a] += fy; F[2 * n + a] += fz; }
        if (dEdrho)
            dEdrho[a] = G[a] * R[a] * R[a] * (1.0 / (rta * rta) - T[a] / (rho[a] * rho[a]))
                      + B[a] * (I[a] + rta * drt_sum) + screen[a] * dS_sum;
    }
    if (Gout) memcpy(Gout, G, sizeof(double) * n);
    if (Rout) memcpy(Rout, R, sizeof(double) * n);
    free(I); free(R); free(T); free(dRdPsi); free(G); free(B);
}

/* ------------------------------------------------------------------------
 * Sites of one system.  Atom indices are local to the system.
 *   site_atom_offset[S+1] -> site_atoms;  site_state_offset[S+1] -> states;
 *   state_charge_offset[n_states_total+1] -> state_charges (one row of
 *   |A_m| charges per state, in the order of the site's atoms).
 * Candidates: sites in index order; within a site every state s' != s in
 * ascending order.
 * ------------------------------------------------------------------------ */

static double pair_K(const double* x, const double* y, const double* z, const double* R,
                     const or_params* p, int i, int k)
{
    double kk = p->coulomb_k;
    if (i == k) return -kk * gb_d(p, R[i]) / R[i];
    double r = dist(x, y, z, i, k), f, ex, D;
    if (beyond(p, r)) return 0.0;
    fgb(r, R[i], R[k], &f, &ex, &D);
    return kk / (p->eps_in * r) - kk * gb_d(p, f) / f;
}

/* Delta E_elec of one candidate, bilinear form: dq.phi + 1/2 dq.K.dq
 * (E is quadratic in q at fixed coordinates and Born radii). */
static double cand_dE(const double* x, const double* y, const double* z, const double* R,
                      const double* phi, const or_params* p, const int* atoms, int na,
                      const double* q_new, const double* q_old)
{
    double lin = 0.0, quad = 0.0;
    for (int a = 0; a < na; ++a) {
        double dqa = q_new[a] - q_old[a];
        lin += dqa * phi[atoms[a]];
        for (int b = 0; b < na; ++b)
            quad += dqa * (q_new[b] - q_old[b]) * pair_K(x, y, z, R, p, atoms[a], atoms[b]);
    }
    return lin + 0.5 * quad;
}

int or_count_candidates(int n_sites, const int* site_state_offset)
{
    int c = 0;
    for (int m = 0; m < n_sites; ++m) c += site_state_offset[m + 1] - site_state_offset[m] - 1;
    return c;
}

void or_site_dE(int n, const double* x, const double* y, const double* z, const double* q,
                const double* R, const or_params* p, int n_sites, const int* site_atom_offset,
                const int* site_atoms, const int* site_state_offset,
                const int* state_charge_offset, const double* state_charges,
                const int* current_state, double* dE)
{
    double* phi = malloc(sizeof(double) * n);
    or_phi_fixedR(n, x, y, z, q, R, p, phi);
    int c = 0;
    for (int m = 0; m < n_sites; ++m) {
        const int* atoms = site_atoms + site_atom_offset[m];
        int na = site_atom_offset[m + 1] - site_atom_offset[m];
        int g0 = site_state_offset[m], ns = site_state_offset[m + 1] - g0;
        const double* qs = state_charges + state_charge_offset[g0 + current_state[m]];
        for (int t = 0; t < ns; ++t) {
            if (t == current_state[m]) continue;
            dE[c++] = cand_dE(x, y, z, R, phi, p, atoms, na,
                              state_charges + state_charge_offset[g0 + t], qs);
        }
    }
    free(phi);
}

/* The same candidates by brute force: E(q') - E(q) with every other charge
 * held at its current value. */
void or_site_dE_brute(int n, const double* x, const double* y, const double* z,
                      const double* q, const double* R, const or_params* p, int n_sites,
                      const int* site_atom_offset, const int* site_atoms,
                      const int* site_state_offset, const int* state_charge_offset,
                      const double* state_charges, const int* current_state, double* dE)
{
    double e0[2], e1[2];
    double* qq = malloc(sizeof(double) * n);
    or_energy_fixedR(n, x, y, z, q, R, p, e0);
    int c = 0;
    for (int m = 0; m < n_sites; ++m) {
        const int* atoms = site_atoms + site_atom_offset[m];
        int na = site_atom_offset[m + 1] - site_atom_offset[m];
        int g0 = site_state_offset[m], ns = site_state_offset[m + 1] - g0;
        for (int t = 0; t < ns; ++t) {
            if (t == current_state[m]) continue;
            memcpy(qq, q, sizeof(double) * n);
            const double* qs = state_charges + state_charge_offset[g0 + t];
            for (int a = 0; a < na; ++a) qq[atoms[a]] = qs[a];
            or_energy_fixedR(n, x, y, z, qq, R, p, e1);
            dE[c++] = (e1[0] + e1[1]) - (e0[0] + e0[1]);
        }
    }
    free(qq);
}

/* Delta G of moving a site from state s to s' (Eq. 8 for redox, Eq. 9 for
 * protonation, in their multi-state form):
 *   protonation: dE + kB T ln10 pH (n_H(s') - n_H(s)) - (Gref(s') - Gref(s))
 *   redox:       dE + F E       (n_e(s') - n_e(s)) - (Gref(s') - Gref(s))
 * With two states, Gref(prot) - Gref(deprot) = dG_elec,ref + kB T ln10 pKa,ref
 * and Gref(red) - Gref(oxi) = dG_elec,ref + F E0_ref reproduce Eqs. 9 and 8. */
double or_delta_G(int kind, double dE, int n_new, int n_old, double gref_new, double gref_old,
                  double pH, double E_volt, double T)
{
    double drive = (kind == 0) ? OR_KB * T * OR_LN10 * pH : OR_FARADAY * E_volt;
    return dE + drive * (double)(n_new - n_old) - (gref_new - gref_old);
}

/* Metropolis: accept iff u < exp(-dG / (kB T)). */
int or_metropolis(double dG, double T, double u)
{
    return u < exp(-dG / (OR_KB * T));
}

static int pick(double u, int n)
{
    int k = (int)floor(u * n);
    return k < n - 1 ? k : n - 1;
}

/* One implicit-solvent C(pH,E)MD attempt pair on one system (Fig. 1 and
 * section III.A.1): a protonation attempt on one protonation site picked
 * uniformly, then a redox attempt on one redox site picked uniformly, which
 * sees the charges left by the protonation attempt.  The proposed state is
 * drawn uniformly from the site's other states.  u[6]: site pick, state pick
 * and acceptance uniform for protonation, then the same for redox.
 * q and current_state are updated in place.  out[4] = {accepted_prot,
 * accepted_redox, cand_prot, cand_redox} (candidate index or -1);
 * out_dG[2] = the two Delta G values (0 when no attempt). */
void or_mc_step(int n, const double* x, const double* y, const double* z, double* q,
                const double* R, const or_params* p, int n_sites, const int* site_kind,
                const int* site_atom_offset, const int* site_atoms, const int* site_state_offset,
                const int* state_charge_offset, const double* state_charges,
                const double* state_gref, const int* state_count, int* current_state,
                double pH, double E_volt, double T, const double* u, int* out, double* out_dG)
{
    double* phi = malloc(sizeof(double) * n);
    out[0] = out[1] = 0;
    out[2] = out[3] = -1;
    out_dG[0] = out_dG[1] = 0.0;
    for (int pass = 0; pass < 2; ++pass) {
        int kind = pass == 0 ? 0 : 1;
        int cnt = 0;
        for (int m = 0; m < n_sites; ++m) cnt += site_kind[m] == kind;
        if (cnt == 0) continue;
        int which = pick(u[3 * pass + 0], cnt), m = -1;
        for (int mm = 0; mm < n_sites; ++mm)
            if (site_kind[mm] == kind && which-- == 0) { m = mm; break; }
        int g0 = site_state_offset[m], ns = site_state_offset[m + 1] - g0;
        int s = current_state[m];
        int tp = pick(u[3 * pass + 1], ns - 1);
        int s_new = tp < s ? tp : tp + 1;
        int cand = 0;
        for (int mm = 0; mm < m; ++mm) cand += site_state_offset[mm + 1] - site_state_offset[mm] - 1;
        cand += tp;
        /* Delta E at the *current* charges (after any accepted protonation) */
        or_phi_fixedR(n, x, y, z, q, R, p, phi);
        const int* atoms = site_atoms + site_atom_offset[m];
        int na = site_atom_offset[m + 1] - site_atom_offset[m];
        const double* q_new = state_charges + state_charge_offset[g0 + s_new];
        const double* q_old = state_charges + state_charge_offset[g0 + s];
        double dE = cand_dE(x, y, z, R, phi, p, atoms, na, q_new, q_old);
        double dG = or_delta_G(kind, dE, state_count[g0 + s_new], state_count[g0 + s],
                               state_gref[g0 + s_new], state_gref[g0 + s], pH, E_volt, T);
        out_dG[pass] = dG;
        out[2 + pass] = cand;
        if (or_metropolis(dG, T, u[3 * pass + 2])) {
            out[pass] = 1;
            current_state[m] = s_new;
            for (int a = 0; a < na; ++a) q[atoms[a]] = q_new[a];
        }
    }
    free(phi);
}

/* One sequential sweep of the explicit-solvent attempt loop (section
 * III.A.2), at fixed coordinates and Born radii: every site of the requested
 * kinds (bit 0 protonation, bit 1 redox) is attempted once; protonation sites
 * come first when both kinds are swept (section III.A), each kind's sites in
 * the random order of ascending u[3m] (ties by index).  Site m proposes the
 * floor(u[3m+1] (n_states - 1))-th of its other states in ascending order and
 * accepts iff u[3m+2] < exp(-dG/(kB T)), with Delta E taken at the charges
 * left by the earlier attempts of the sweep (potentials recomputed from all
 * atoms at every visit).  accepted[m] is 1/0 for attempted sites and -1 for
 * the others; out_dG[m] receives the attempt's Delta G. */
void or_mc_sweep(int n, const double* x, const double* y, const double* z, double* q,
                 const double* R, const or_params* p, int n_sites, const int* site_kind,
                 const int* site_atom_offset, const int* site_atoms, const int* site_state_offset,
                 const int* state_charge_offset, const double* state_charges,
                 const double* state_gref, const int* state_count, int* current_state,
                 double pH, double E_volt, double T, int kinds, const double* u, int* accepted,
                 double* out_dG)
{
    double* phi = malloc(sizeof(double) * n);
    int* order = malloc(sizeof(int) * (n_sites > 0 ? n_sites : 1));
    for (int m = 0; m < n_sites; ++m) { accepted[m] = -1; out_dG[m] = 0.0; }
    for (int kind = 0; kind < 2; ++kind) {
        if (!(kinds & (1 << kind))) continue;
        int cnt = 0;
        for (int m = 0; m < n_sites; ++m)
            if (site_kind[m] == kind) order[cnt++] = m;
        /* insertion sort by (u[3m], m) */
        for (int a = 1; a < cnt; ++a) {
            int m = order[a], b = a - 1;
            while (b >= 0 && (u[3 * order[b]] > u[3 * m] ||
                              (u[3 * order[b]] == u[3 * m] && order[b] > m))) {
                order[b + 1] = order[b];
                --b;
            }
            order[b + 1] = m;
        }
        for (int v = 0; v < cnt; ++v) {
            int m = order[v];
            int g0 = site_state_offset[m], ns = site_state_offset[m + 1] - g0;
            int s = current_state[m];
            int tp = pick(u[3 * m + 1], ns - 1);
            int s_new = tp < s ? tp : tp + 1;
            or_phi_fixedR(n, x, y, z, q, R, p, phi);
            const int* atoms = site_atoms + site_atom_offset[m];
            int na = site_atom_offset[m + 1] - site_atom_offset[m];
            const double* q_new = state_charges + state_charge_offset[g0 + s_new];
            const double* q_old = state_charges + state_charge_offset[g0 + s];
            double dE = cand_dE(x, y, z, R, phi, p, atoms, na, q_new, q_old);
            double dG = or_delta_G(kind, dE, state_count[g0 + s_new], state_count[g0 + s],
                                   state_gref[g0 + s_new], state_gref[g0 + s], pH, E_volt, T);
            out_dG[m] = dG;
            accepted[m] = or_metropolis(dG, T, u[3 * m + 2]);
            if (accepted[m]) {
                current_state[m] = s_new;
                for (int a = 0; a < na; ++a) q[atoms[a]] = q_new[a];
            }
        }
    }
    free(order);
    free(phi);
}

/* n_steps attempt pairs at fixed coordinates and Born radii; u[n_steps][6].
 * occupancy[n_states_total] accumulates, after every step, one count for the
 * state each site is in. */
void or_mc_run(int n_steps, int n, const double* x, const double* y, const double* z,
               double* q, const double* R, const or_params* p, int n_sites, const int* site_kind,
               const int* site_atom_offset, const int* site_atoms, const int* site_state_offset,
               const int* state_charge_offset, const double* state_charges,
               const double* state_gref, const int* state_count, int* current_state,
               double pH, double E_volt, double T, const double* u, int64_t* occupancy,
               int64_t* accepted)
{
    int out[4];
    double dG[2];
    for (int it = 0; it < n_steps; ++it) {
        or_mc_step(n, x, y, z, q, R, p, n_sites, site_kind, site_atom_offset, site_atoms,
                   site_state_offset, state_charge_offset, state_charges, state_gref,
                   state_count, current_state, pH, E_volt, T, u + 6 * (int64_t)it, out, dG);
        accepted[0] += out[0];
        accepted[1] += out[1];
        for (int m = 0; m < n_sites; ++m) occupancy[site_state_offset[m] + current_state[m]]++;
    }
}

/* E-REMD exchange attempt (section II.C and III.B).  Rungs are ordered by
 * redox potential E_rung[M]; rep_of_rung[M] is the replica at each rung.
 * Parity 0 pairs rungs (0,1),(2,3),...; parity 1 pairs (1,2),(3,4),... and,
 * with wrap set and M even, (M-1,0).  For the pair (rung l holding replica i,
 * rung n holding replica j), Delta = F (E_n - E_l)(N_i - N_j) / (kB T)
 * (Eq. 14); accept if Delta < 0 or u < exp(-Delta) (Eq. 15); on acceptance
 * the two replicas swap rungs.  u[p] and accepted[p] are indexed by the pair's
 * position in that list.  E_of_rep[M] receives every replica's redox
 * potential after the attempt.  Returns the number of pairs. */
int or_remd_exchange(int M, const double* E_rung, const int* Ne_of_rep, int* rep_of_rung,
                     double T, int parity, int wrap, const double* u, int* accepted,
                     double* E_of_rep)
{
    int np = 0;
    for (int l = parity; l + 1 < M; l += 2) {
        int n2 = l + 1;
        int i = rep_of_rung[l], j = rep_of_rung[n2];
        double delta = OR_FARADAY * (E_rung[n2] - E_rung[l]) * (double)(Ne_of_rep[i] - Ne_of_rep[j])
                     / (OR_KB * T);
        int acc = delta < 0.0 || u[np] < exp(-delta);
        if (acc) { rep_of_rung[l] = j; rep_of_rung[n2] = i; }
        accepted[np++] = acc;
    }
    if (parity == 1 && wrap && M % 2 == 0 && M > 2) {
        int l = M - 1, n2 = 0;
        int i = rep_of_rung[l], j = rep_of_rung[n2];
        double delta = OR_FARADAY * (E_rung[n2] - E_rung[l]) * (double)(Ne_of_rep[i] - Ne_of_rep[j])
                     / (OR_KB * T);
        int acc = delta < 0.0 || u[np] < exp(-delta);
        if (acc) { rep_of_rung[l] = j; rep_of_rung[n2] = i; }
        accepted[np++] = acc;
    }
    for (int l = 0; l < M; ++l) E_of_rep[rep_of_rung[l]] = E_rung[l];
    return np;
}

/* One leapfrog Langevin step of one system (Loncharich, Brooks & Pastor 1992).
 * With a = gamma dt / 2 and c = OR_ACC (kcal/mol/(amu A) -> A/ps^2), for every
 * atom i and Cartesian component:
 *   F    = -dE_elec/dx_i - k_restr (x_i - xref_i)       (E_elec: Coulomb + GB)
 *   v_i <- [ (1 - a) v_i + dt c F / m_i + sqrt(2 gamma kB T dt c / m_i) xi ]
 *          / (1 + a)
 *   x_i <- x_i + dt v_i
 * v is the half-step velocity v(t - dt/2) on entry and v(t + dt/2) on exit,
 * [3n] component-major, A/ps;  inv_mass[n] in 1/amu (0 with zero velocity
 * holds an atom still);
 * xi[3n] standard normal deviates, component-major;  xref[3n] or NULL (no
 * restraint);  dt in ps, gamma in 1/ps, T in K.  Forces are evaluated at the
 * coordinates on entry with the full FP64 definition (or_energy_forces). */
void or_langevin_step(int n, double* x, double* y, double* z, const double* q,
                      const double* rho, const double* screen, const or_params* p,
                      const double* xref, double k_restr, double* v, const double* inv_mass,
                      const double* xi, double dt, double gamma, double T)
{
    double* F = malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    double E[2];
    or_energy_forces(n, x, y, z, q, rho, screen, p, E, F, NULL, NULL, NULL, NULL);
    double* pos[3] = {x, y, z};
    double a = 0.5 * gamma * dt;
    for (int c = 0; c < 3; ++c) {
        for (int i = 0; i < n; ++i) {
            double f = F[c * n + i];
            if (xref) f -= k_restr * (pos[c][i] - xref[c * n + i]);
            double im = inv_mass[i];
            double sig = sqrt(2.0 * gamma * OR_KB * T * dt * OR_ACC * im);
            double vi = ((1.0 - a) * v[c * n + i] + dt * OR_ACC * f * im + sig * xi[c * n + i])
                      / (1.0 + a);
            v[c * n + i] = vi;
            pos[c][i] += dt * vi;
        }
    }
    free(F);
}
