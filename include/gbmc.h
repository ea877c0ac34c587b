/*
 * gbmc.h -- C ABI of libgbmc: all-pairs Generalized Born (OBC) electrostatics
 * and the discrete-state Monte Carlo / replica-exchange decisions of constant
 * redox potential MD (CEMD), coupled constant pH and redox potential MD
 * (C(pH,E)MD) and redox potential replica exchange MD (E-REMD) in implicit
 * solvent, after Cruzeiro, Amaral & Roitberg, arXiv:1803.09652, on AMD
 * Instinct MI355X (gfx950).
 *
 * Conventions
 *  - Units: Angstrom, elementary charge, kcal/mol, volt, kelvin.
 *  - Every array argument is a DEVICE pointer owned by the caller unless its
 *    comment says "host".  The library never frees caller memory.
 *  - Every compute call is asynchronous on the caller's stream, performs no
 *    host<->device synchronisation and no allocation, and may be captured in a
 *    HIP graph (accumulators are cleared by kernels, never by memset).
 *  - Every call returns a gbmc_status; on failure gbmc_last_error() returns a
 *    thread-local message.  No C++ exception crosses this interface.
 *  - A plan fixes the batch layout (systems of uneven size, concatenated) and
 *    the precision.  In GBMC_FP32_FIXED plans per-atom arrays are float, pair
 *    arithmetic is FP32 and every sum is accumulated in 64-bit fixed point, so
 *    results are bitwise reproducible run to run; in GBMC_FP64 plans per-atom
 *    arrays are double and the arithmetic is FP64.  Arrays documented as
 *    double are FP64 in both precisions.
 *  - Coordinates must lie within +-1e5 A and no two atoms of a system may
 *    coincide (r_ij > 0).
 */
#ifndef GBMC_H
#define GBMC_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GBMC_OK = 0,
    GBMC_ERR_INVALID = -1,      /* bad argument, layout or table */
    GBMC_ERR_HIP = -2,          /* a HIP runtime call failed */
    GBMC_ERR_OVERFLOW = -3,     /* a fixed-point accumulator would overflow */
    GBMC_ERR_UNSUPPORTED = -4   /* valid input this library does not handle */
} gbmc_status;

typedef enum { GBMC_FP32_FIXED = 0, GBMC_FP64 = 1 } gbmc_precision;

/* GB model parameters.  The paper runs the Onufriev-Bashford-Case model with
 * AMBER's igb=2 set (section III.D/E: alpha 0.8, beta 0, gamma 2.909125); the
 * igb=5 set is alpha 1.0, beta 0.8, gamma 4.85.  offset is the dielectric
 * offset subtracted from every intrinsic radius (0.09 A); coulomb_k is the
 * Coulomb constant (332.0522 kcal A / (mol e^2)); kappa >= 0 is the inverse
 * Debye length (1/A) of added salt (the paper's runs have none: kappa = 0).
 * With salt every GB pair and self term carries the Debye-Hueckel factor
 * 1/eps_in - exp(-kappa f)/eps_out in place of 1/eps_in - 1/eps_out
 * (Srinivasan et al., Theor. Chem. Acc. 101 (1999) 426).
 * Optional cutoffs for large systems (0 = none, the paper's setting):
 * rgbmax > 0 restricts each atom's descreening integral to the sphere of that
 * radius around it (the part of ball j inside rgbmax and outside rt:
 * H(r; rt, S) - H(r; rgbmax, S)); cutoff > 0 drops the Coulomb and GB pair
 * terms of every pair at or beyond that distance (self terms stay), in the
 * energies, forces, dE/dq, dE/drho and the Monte Carlo Delta E alike.  Tiles
 * of 64 x 64 atoms whose bounding spheres are farther apart are skipped.
 * gb_radii and gb_energy_forces must get the same parameters. */
typedef struct {
    double alpha, beta, gamma;
    double offset;
    double eps_in, eps_out;
    double coulomb_k;
    double kappa;
    double rgbmax;
    double cutoff;
} gbmc_gb_params;

/* Per-atom SoA inputs over the whole batch (N_tot = atom_offset[B] atoms),
 * element type float (FP32_FIXED plans) or double (FP64 plans):
 * x, y, z coordinates; q partial charges; rho intrinsic GB radii (> offset);
 * screen HCT screening factors (>= 0). */
typedef struct {
    const void* x;
    const void* y;
    const void* z;
    const void* q;
    const void* rho;
    const void* screen;
} gbmc_atoms;

/* Work-shape knobs of the three pair passes (index GBMC_PASS_*): how many
 * 64-atom j blocks one wavefront walks for its i block (>= 1), and how many
 * such independent wavefronts share a workgroup (1, 2, 4 or 8).  Every 64 x 64
 * tile is rounded into fixed point on its own, so results are bitwise
 * independent of the knobs.  Defaults (tuning NULL; j blocks / waves): FP32
 * descreening 1 / 2, energy 1 / 4, chain 1 / 4, and for FP32 batches of at
 * least 2^19 tiles (sum over systems of nb (nb + 1) / 2, nb = ceil(n / 64))
 * energy and chain 4 / 1; FP64 1 / 2 for all three passes. */
enum { GBMC_PASS_RADII = 0, GBMC_PASS_ENERGY = 1, GBMC_PASS_CHAIN = 2, GBMC_N_PASSES = 3 };
typedef struct {
    int32_t j_blocks_per_item[GBMC_N_PASSES];
    int32_t waves_per_group[GBMC_N_PASSES];
} gbmc_tuning;

typedef struct gbmc_plan gbmc_plan;
typedef struct gbmc_sites gbmc_sites;

/* Library version (major * 10000 + minor * 100 + patch). */
int32_t gbmc_version(void);

/* Thread-local message describing the last failure of this thread. */
const char* gbmc_last_error(void);

/* Host-only check of GB parameters: GBMC_ERR_INVALID for kappa < 0,
 * rgbmax < 0, cutoff < 0, eps_in <= 0, eps_out <= 0, offset < 0 or non-finite
 * values. */
gbmc_status gbmc_params_validate(const gbmc_gb_params* params);

/* Host-only: the pair-tile work list a plan with this layout would use for a
 * pass walking j_blocks_per_item j blocks per item (>= 1); row_pairs != 0
 * gives the schedule of the FP32 plans' energy and chain passes, 0 that of
 * their descreening pass and of every pass of FP64 plans.
 * host_atom_offset[n_systems+1] (host) must start at 0 and be non-decreasing.
 * Each item covers, for one system, the 64-atom i blocks [I0, I1) (one or
 * two) against the j blocks [J0, J1), J0 >= I0 (every unordered pair of atoms
 * lies in exactly one tile, the diagonal tile I == J holding the pairs inside
 * one block).  With row_pairs the i blocks are paired (2a, 2a + 1): two-row
 * items cover the pair against J >= 2a + 2, one-row items the diagonal band
 * and an unpaired last block; without, every item has one i block.  Items are
 * ordered by decreasing cost.  *n_items receives the count; if items (host) is
 * not NULL it receives 5 int32 per item: system, I0, I1, J0, J1 (the caller
 * sizes it from a first call with items == NULL). */
gbmc_status gbmc_schedule_build(int32_t n_systems, const int32_t* host_atom_offset,
                                int32_t j_blocks_per_item, int32_t row_pairs, int32_t* n_items,
                                int32_t* items);

/* Host-only: the work sequence of the queued single launch
 * (gbmc_plan_set_single_launch) that a plan with this layout, precision and
 * tuning (NULL: the defaults) runs, for checking its ordering off the GPU.
 * n_items[3] (host) receives the item count of each pass; *n_blocks the number
 * of 64-atom blocks of the batch (per system ceil(n / 64), systems in order).
 * If items (host, 7 int32 per item, sized from a first call with items ==
 * NULL) is not NULL it receives the items in sequence order (the descreening
 * pass's, then the energy pass's, then the chain pass's): pass, system, index
 * of the system's first block, I0, I1, J0, J1 (the tiles of i blocks [I0, I1)
 * against j blocks [J0, J1), as in gbmc_schedule_build).  If totals (host,
 * [3][n_blocks]) is not NULL it receives the number of items of each pass that
 * touch each block: the counts at which the launch's per-block counters mark a
 * block final for that pass.  GBMC_ERR_INVALID for bad offsets, precision or
 * tuning, as gbmc_plan_create. */
gbmc_status gbmc_queue_schedule(int32_t n_systems, const int32_t* host_atom_offset,
                                gbmc_precision precision, const gbmc_tuning* tuning,
                                int32_t* n_items, int32_t* items, int32_t* n_blocks,
                                int32_t* totals);

/* Create a plan for a batch of n_systems systems laid out back to back:
 * system b owns atoms [host_atom_offset[b], host_atom_offset[b+1]) (host array,
 * copied).  Empty systems are allowed.  tuning may be NULL (defaults).  The
 * plan allocates its own device copy of the work list (the only device
 * allocation the library makes, here and in gbmc_sites_create).  Requires the
 * HIP device the plan will run on to be current. */
gbmc_status gbmc_plan_create(gbmc_plan** plan, int32_t n_systems, const int32_t* host_atom_offset,
                             gbmc_precision precision, const gbmc_tuning* tuning);
void gbmc_plan_destroy(gbmc_plan* plan);

/* Processing order (staging).  Every pair pass first packs the atoms of each
 * system into the workspace in the plan's processing order; an order that
 * keeps nearby atoms together confines the overlapping pairs (which take the
 * slow branch of the descreening integral) to few tiles.  host_order (host,
 * N_tot entries, copied) lists for every internal position the caller atom
 * index processed there and must be a permutation of each system's atom range.
 * Outputs are always in caller order; results depend on the order only
 * through FP32 rounding inside tiles (bitwise reproducible for a given order).
 * The default is the identity.  Synchronous (not graph-capturable). */
gbmc_status gbmc_plan_set_order(gbmc_plan* plan, const int32_t* host_order);

/* Host-only helper: a spatial (Morton, 10 bits per axis) order of each
 * system's atoms from host coordinates x, y, z [N_tot] (double), written to
 * order[N_tot] for gbmc_plan_set_order. */
gbmc_status gbmc_spatial_order(int32_t n_systems, const int32_t* host_atom_offset, const double* x,
                               const double* y, const double* z, int32_t* order);

/* Host-only helper: an order of each system's atoms in which every 64-atom
 * block is a compact cluster, by recursive bisection along the longest side
 * of the bounding box with every cut after a multiple of 64 atoms (ties by
 * index).  Compact blocks have small bounding spheres, so the cutoff passes
 * visit fewer tiles.  Same arguments as gbmc_spatial_order. */
gbmc_status gbmc_block_order(int32_t n_systems, const int32_t* host_atom_offset, const double* x,
                             const double* y, const double* z, int32_t* order);

/* Bytes of caller-owned device workspace a plan needs (256-byte aligned).
 * The workspace carries per-atom state from gb_radii to gb_energy_forces and
 * mc_state_dE; one workspace may serve one stream at a time. */
size_t gbmc_plan_workspace_bytes(const gbmc_plan* plan);

/* Effective Born radii (the GB model of section III.D; OBC formula):
 *   I_i = sum_{j != i} H(r_ij; rho_i - offset, screen_j (rho_j - offset))
 *   Psi_i = (rho_i - offset) I_i,  theta = alpha Psi - beta Psi^2 + gamma Psi^3
 *   R_i = 1 / (1/(rho_i - offset) - tanh(theta)/rho_i)
 * where H is the HCT pair integral, restricted to the sphere of radius
 * params->rgbmax around atom i when rgbmax > 0 (see gbmc_gb_params).  Writes born_R[N_tot] (float or
 * double per plan) and the per-atom state that gb_energy_forces and
 * mc_state_dE use into workspace. */
gbmc_status gb_radii(gbmc_plan* plan, const gbmc_atoms* atoms, const gbmc_gb_params* params,
                     void* workspace, void* born_R, hipStream_t stream);

/* Coulomb + GB energy and its derivatives, the electrostatics of the MD steps
 * between Monte Carlo attempts (section III.A, Fig. 1):
 *   E_C  = k sum_{i<j} q_i q_j / (eps_in r_ij)
 *   E_GB = -(k/2) sum_i sum_j q_i q_j d(f_ij) / f_ij,
 *   f_ij = sqrt(r^2 + R_i R_j exp(-r^2 / (4 R_i R_j))),  f_ii = R_i,
 *   d(f) = 1/eps_in - exp(-kappa f)/eps_out  (1/eps_in - 1/eps_out without salt),
 * using the radii of the preceding gb_radii call on the same workspace and
 * atoms.  Outputs (each may be NULL):
 *   e_coul[B], e_gb[B]  double, per system;
 *   force[N_tot][3]     -dE/dx including the Born-radius chain term;
 *   dEdq[N_tot]         dE/dq (electrostatic potential, self term included);
 *   dEdrho[N_tot]       dE/drho at fixed screening factors.
 * With force, dEdq and dEdrho all NULL only the energies are computed. */
gbmc_status gb_energy_forces(gbmc_plan* plan, const gbmc_atoms* atoms,
                             const gbmc_gb_params* params, void* workspace,
                             double* e_coul, double* e_gb, void* force, void* dEdq,
                             void* dEdrho, hipStream_t stream);

/* One full evaluation: gb_radii followed by gb_energy_forces on the same
 * workspace (Born radii from the geometry, section III.D; the electrostatic
 * energy and its derivatives of the MD steps, section III.A, Fig. 1), with the
 * inputs staged once for all passes.  Outputs and their layout as in those
 * two calls, bitwise the same (born_R may be NULL; the energies and gradients
 * as in gb_energy_forces).  Leaves the per-atom state in workspace for
 * mc_state_dE, mc_step and mc_sweep. */
gbmc_status gb_evaluate(gbmc_plan* plan, const gbmc_atoms* atoms, const gbmc_gb_params* params,
                        void* workspace, void* born_R, double* e_coul, double* e_gb, void* force,
                        void* dEdq, void* dEdrho, hipStream_t stream);

/* gb_evaluate that also hands the Born radii to a second stream as soon as
 * they are final: the call records an event of the plan on `stream` after the
 * radii pass and its finalize and makes `fork` wait on it (hipStreamWaitEvent),
 * then issues the energy and force passes on `stream`.  Work the caller queues
 * on `fork` after the call (mc_state_dE, mc_step: the Monte Carlo attempt of
 * Fig. 1, which needs the radii and the charges only) then overlaps the energy
 * and force passes; both streams may be under one hipGraph capture.  Outputs
 * as in gb_evaluate, bitwise the same as gb_radii + gb_energy_forces.  Work on
 * `fork` must not write the atoms' inputs or the workspace's pass
 * accumulators before it rejoins `stream`.  GBMC_ERR_INVALID if fork equals
 * stream; GBMC_ERR_HIP if the event record or wait fails.  Calls on one plan
 * share its event: calls that may overlap (several streams, several threads)
 * must be ordered by the caller. */
gbmc_status gb_evaluate_fork(gbmc_plan* plan, const gbmc_atoms* atoms,
                             const gbmc_gb_params* params, void* workspace, void* born_R,
                             double* e_coul, double* e_gb, void* force, void* dEdq, void* dEdrho,
                             hipStream_t stream, hipStream_t fork);

/* gb_evaluate without a caller workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the workspace is a library-owned static array of
 * 256 MiB per GPU (held until the process ends), so the call itself allocates
 * nothing.  Inputs and outputs are the caller's, as in gb_evaluate.
 * GBMC_ERR_UNSUPPORTED if the plan needs a larger workspace than that
 * (gbmc_plan_workspace_bytes); GBMC_ERR_HIP if the array's device address
 * could not be obtained when the plan was created.  Every call on one GPU
 * shares that GPU's array and leaves its per-atom state there (each call
 * clears what must start at zero): calls that may overlap on one GPU (other
 * streams, other threads, other plans) race and must be serialised by the
 * caller, and the state is not meant for mc_state_dE.  The overflow flag of
 * these calls is read with gbmc_check_overflow(plan, NULL, ...). */
gbmc_status gb_evaluate_static(gbmc_plan* plan, const gbmc_atoms* atoms,
                               const gbmc_gb_params* params, void* born_R, double* e_coul,
                               double* e_gb, void* force, void* dEdq, void* dEdrho,
                               hipStream_t stream);

/* The plain FP64 GPU form of one full evaluation: the same outputs as
 * gb_radii + gb_energy_forces of an FP64 plan (radii born_R[N], e_coul[B],
 * e_gb[B], force[N][3], dEdq[N], dEdrho[N]; each may be NULL) computed the
 * direct way, one thread per atom over its whole row (every ordered pair),
 * closed forms with correctly rounded division, square root, exp and log.  It
 * is the reference the pair rate of the batched forms is compared with.
 * Needs no plan: host_atom_offset (host) and atom_offset (device) [B+1]; all
 * arrays double, caller order; workspace of gb_plain_workspace_bytes(N)
 * bytes (caller-owned, device).  No salt and no cutoffs
 * (GBMC_ERR_UNSUPPORTED). */
size_t gb_plain_workspace_bytes(int32_t n_atoms);
gbmc_status gb_plain_fp64(int32_t n_systems, const int32_t* host_atom_offset,
                          const int32_t* atom_offset, const gbmc_atoms* atoms,
                          const gbmc_gb_params* params, void* workspace, double* born_R,
                          double* e_coul, double* e_gb, double* force, double* dEdq,
                          double* dEdrho, hipStream_t stream);

/* Titratable sites (host arrays, copied to the device; sites of one system
 * must be disjoint):
 *   site_system[S]          system of each site (non-decreasing)
 *   site_kind[S]            0 = protonation, 1 = redox
 *   site_atom_offset[S+1]   CSR into site_atoms (1..256 atoms per site)
 *   site_atoms[...]         global atom indices inside the site's system
 *   site_state_offset[S+1]  CSR into the state tables (2..8 states per site)
 *   state_charge_offset[n_states_total+1] CSR into state_charges; row g holds
 *                           the site's atom charges in state g
 *   state_charges[...]      double
 *   state_gref[n_states_total] double, kcal/mol: reference free energy of each
 *                           state; for two states Gref(red) - Gref(oxi) =
 *                           dG_elec,ref + F E0_ref (Eq. 8) and Gref(prot) -
 *                           Gref(deprot) = dG_elec,ref + kB T ln10 pKa,ref (Eq. 9)
 *   state_count[n_states_total]  protons n_H (protonation) or electrons n_e
 *                           (redox) of each state.
 * Candidates: every site in index order, and within a site every state other
 * than the current one in ascending order; sites_n_candidates is their count. */
gbmc_status gbmc_sites_validate(int32_t n_systems, const int32_t* host_atom_offset,
                                int32_t n_sites, const int32_t* site_system,
                                const int32_t* site_kind, const int32_t* site_atom_offset,
                                const int32_t* site_atoms, const int32_t* site_state_offset,
                                const int32_t* state_charge_offset, const int32_t* state_count);
gbmc_status gbmc_sites_create(gbmc_plan* plan, gbmc_sites** sites, int32_t n_sites,
                              const int32_t* site_system, const int32_t* site_kind,
                              const int32_t* site_atom_offset, const int32_t* site_atoms,
                              const int32_t* site_state_offset,
                              const int32_t* state_charge_offset, const double* state_charges,
                              const double* state_gref, const int32_t* state_count);
void gbmc_sites_destroy(gbmc_sites* sites);
int32_t gbmc_sites_n_candidates(const gbmc_sites* sites);
/* Bytes of caller-owned device workspace mc_state_dE and mc_step need: the
 * site atoms' FP64 potentials as int64 fixed point (2^-44 kcal/mol/e), which
 * mc_state_dE clears and fills on every call. */
size_t gbmc_sites_workspace_bytes(const gbmc_sites* sites);

/* Delta E_elec and Delta G of every candidate state change (sections II.A-B):
 * the electrostatic energy difference between the proposed and the current
 * state at fixed coordinates and Born radii, in FP64,
 *   dE = dq . phi + 1/2 dq . K . dq,   dq = Q_m[s'] - Q_m[s] on the site atoms,
 * and
 *   protonation: dG = dE + kB T ln10 pH[b] (n_H(s') - n_H(s)) - (Gref(s') - Gref(s))
 *   redox:       dG = dE + F E_volt[b] (n_e(s') - n_e(s)) - (Gref(s') - Gref(s)),
 * the multi-state form of Eqs. 9 and 8.  current_state[S] (int32), pH[B] and
 * E_volt[B] (double) are device arrays; dE_elec and dG receive n_candidates
 * doubles (dG may be NULL).  Uses the coordinates and Born radii of the last
 * gb_radii call on workspace: atoms must hold those coordinates, and atoms->q
 * the charges of current_state. */
gbmc_status mc_state_dE(gbmc_plan* plan, const gbmc_sites* sites, const gbmc_atoms* atoms,
                        const gbmc_gb_params* params, void* workspace, void* site_workspace,
                        const int32_t* current_state, const double* pH, const double* E_volt,
                        double T, double* dE_elec, double* dG, hipStream_t stream);

/* One implicit-solvent C(pH,E)MD attempt pair per system (section III.A.1,
 * Fig. 1): a protonation attempt on one protonation site picked uniformly,
 * then a redox attempt on one redox site picked uniformly; each proposes one
 * of the site's other states uniformly and accepts iff u < exp(-dG/(kB T))
 * (Metropolis, FP64).  The redox attempt sees the charges left by an accepted
 * protonation attempt: its dG gains dq_redox . K . dq_prot.  Inputs dE_elec
 * and dG come from mc_state_dE on the same state.  u[B][6] (double, device):
 * site pick, state pick, acceptance for protonation, then for redox; a pick
 * takes floor(u * count) clamped to count - 1.  Updates q[N_tot] (float or
 * double per plan) and current_state[S] in place.  Optional outputs:
 * n_electrons[B] (int32) sum of n_e over each system's redox sites after the
 * step; counters[S][2] (int64) attempts and acceptances added per site;
 * accepted[B][2] (int32) per system flags for the two attempts. */
gbmc_status mc_step(gbmc_plan* plan, const gbmc_sites* sites, const gbmc_atoms* atoms, void* q,
                    const gbmc_gb_params* params, void* workspace, void* site_workspace,
                    int32_t* current_state, const double* pH, const double* E_volt, double T,
                    const double* dE_elec, const double* dG, const double* u,
                    int32_t* n_electrons, int64_t* counters, int32_t* accepted,
                    hipStream_t stream);

/* One sequential Monte Carlo sweep per system: the explicit-solvent attempt
 * loop of section III.A.2 run on the implicit-solvent energies.  Every site
 * of the requested kinds (bit 0 of kinds: protonation, bit 1: redox) is
 * attempted once; protonation sites come first when both kinds are swept
 * (section III.A), each kind's sites of a system in the random order of
 * ascending u[3m] (ties by site index).  Site m proposes the
 * floor(u[3m+1] (n_states - 1))-th of its other states (clamped) and accepts
 * iff u[3m+2] < exp(-dG/(kB T)), with dG as in mc_state_dE taken at the
 * charges left by the earlier attempts of the sweep (FP64).  u[S][3] (double,
 * device).  Accepted site charges are written into q (float or double per
 * plan, may alias atoms->q; the other charges must already be there) and
 * current_state[S] is updated in place.  Optional outputs: n_electrons[B]
 * (int32) after the sweep, counters[S][2] (int64) attempts and acceptances
 * added per site, accepted[S] (int32) 1/0 for the sites attempted (others
 * untouched), dG[S] (double) of each attempt.  Needs the coordinates and Born
 * radii of the last gb_radii call on workspace (atoms must hold them, and
 * atoms->q the charges of current_state).  GBMC_ERR_UNSUPPORTED if a system
 * has more than 1024 site atoms or more than 1024 sites of one kind. */
gbmc_status mc_sweep(gbmc_plan* plan, const gbmc_sites* sites, const gbmc_atoms* atoms, void* q,
                     const gbmc_gb_params* params, void* workspace, void* site_workspace,
                     int32_t* current_state, const double* pH, const double* E_volt, double T,
                     int32_t kinds, const double* u, int32_t* n_electrons, int64_t* counters,
                     int32_t* accepted, double* dG, hipStream_t stream);

/* One leapfrog Langevin step of every atom of the plan (Loncharich, Brooks &
 * Pastor, Biopolymers 32 (1992) 523): the constant-charge dynamics between
 * Monte Carlo attempts, with the Langevin thermostat of section III.D.  With
 * a = gamma dt / 2, for atom i and component c:
 *   F  = force[i][c] - k_restr (x_c - xref[c][i])    (restraint if xref given)
 *   v' = [(1 - a) v + dt 418.4 F / m + sqrt(2 gamma kB T dt 418.4 / m) xi[c][i]]
 *        / (1 + a)
 *   x' = x + dt v'
 * Units: Angstrom, ps, amu, kcal/mol (418.4 converts kcal/mol/(amu A) into
 * A/ps^2).  x, y, z[N_tot] (positions, updated in place), v[3][N_tot]
 * (half-step velocities v(t - dt/2) in, v(t + dt/2) out, A/ps), force[N_tot][3]
 * (the force output of gb_energy_forces at x, or any force), inv_mass[N_tot]
 * (1/amu; 0 with zero velocity holds an atom still), xi[3][N_tot] (standard normal deviates,
 * drawn by the caller), xref[3][N_tot] (restraint centres, NULL for none):
 * device arrays of the plan's float type, caller order; arithmetic in FP64.
 * dt > 0 (ps), gamma >= 0 (1/ps), T >= 0 (K), k_restr >= 0 (kcal/mol/A^2).
 * force must not alias x, y, z or v. */
gbmc_status md_langevin_step(gbmc_plan* plan, void* x, void* y, void* z, void* v,
                             const void* force, const void* inv_mass, const void* xi,
                             const void* xref, double k_restr, double dt, double gamma, double T,
                             hipStream_t stream);

/* E-REMD exchange attempt (section II.C, Eqs. 14-15; pairing of section
 * III.B).  Rungs 0..M-1 are ordered by increasing redox potential E_rung[M]
 * (double, volt); rep_of_rung[M] (int32, in/out) holds the replica at each
 * rung.  parity 0 pairs rungs (0,1),(2,3),...; parity 1 pairs (1,2),(3,4),...
 * and, when wrap is nonzero and M is even and > 2, also (M-1, 0).  For the
 * pair (rung l holding replica i, rung n holding replica j):
 *   Delta = F (E_n - E_l)(N_i - N_j) / (kB T)
 * and the pair swaps rungs iff Delta < 0 or u[p] < exp(-Delta).  Ne_of_rep[M]
 * (int32) are electron counts, u[p] (double) and accepted[p] (int32) are
 * indexed by the pair's position in the list above.  E_of_rep[M] (double,
 * output) receives every replica's redox potential after the attempt.
 * Replicas at different pH form separate ladders and separate calls. */
gbmc_status remd_exchange(int32_t n_rep, const double* E_rung, const int32_t* Ne_of_rep,
                          int32_t* rep_of_rung, double T, int32_t parity, int32_t wrap,
                          const double* u, int32_t* accepted, double* E_of_rep,
                          hipStream_t stream);

/* Single-launch mode of gb_evaluate (off by default).  With enable != 0 a
 * full evaluation without cutoffs (forces or dE/drho requested) runs its three
 * pair passes as one kernel launch instead of one launch per pass.  Its work
 * items form one sequence in pass order; each workgroup takes the next ticket
 * from a device counter when it starts and runs the items of that ticket, so
 * items start in sequence order.  An item of the energy or chain pass first
 * waits until the 64-atom blocks it reads are final in the preceding pass
 * (per-block completion counters; the wave that completes a block finalizes
 * it).  Such a wait only ever waits for items that started earlier, so it
 * ends; it is bounded all the same, by wait_polls polls (each about a
 * microsecond; 0 with enable != 0: give up at once, which forces the failure
 * path in tests; 0 with enable == 0 keeps the current bound; the default is
 * 4194304, seconds, far beyond any wait the schedule produces).  A wave whose
 * wait gives up sets the error flag that gbmc_check_overflow reports, and the
 * launch drains without computing the remaining items.  Results are bitwise
 * those of the separate launches.  On the MI355X the separate launches are
 * faster (the same-address ticket counter and the wait for each item's
 * fixed-point atomics before it counts itself done cost more than the
 * overlap of the passes gains), hence the default. */
gbmc_status gbmc_plan_set_single_launch(gbmc_plan* plan, int32_t enable, int32_t wait_polls);

/* Kernel timing hook (tracing).  While enabled, every compute call on this
 * plan launches each kernel of the hot path with a start and a stop HIP event
 * bound to the dispatch itself (hipExtLaunchKernelGGL), so that their interval
 * is the kernel's own execution, without host synchronisation between calls.
 * gbmc_plan_kernel_ms waits for the last recorded events and writes, per
 * kernel, the mean duration (ms) over its launches since the previous read or
 * the enabling call (the most recent 256 when there were more) into
 * ms[GBMC_N_KERNELS], -1 for kernels not launched; the read starts a new
 * count.  For eager calls only: disable it before capturing a graph. */
enum {
    GBMC_K_RADII_PAIRS = 0,    /* descreening pair pass of gb_radii */
    GBMC_K_ENERGY_PAIRS = 1,   /* energy / explicit force pair pass */
    GBMC_K_CHAIN_PAIRS = 2,    /* Born-radius chain pair pass */
    GBMC_K_SITE_ROWS = 3,      /* FP64 potential rows of mc_state_dE */
    GBMC_K_SITE_DE = 4,        /* per-site Delta E / Delta G of mc_state_dE */
    GBMC_K_MC_STEP = 5,        /* Metropolis step */
    GBMC_K_FORCE_PAIRS = 6,    /* (reserved) */
    GBMC_K_EVAL_PAIRS = 7,     /* single launch of all three passes (gb_evaluate) */
    GBMC_N_KERNELS = 8
};
gbmc_status gbmc_plan_set_timing(gbmc_plan* plan, int32_t enable);
gbmc_status gbmc_plan_kernel_ms(gbmc_plan* plan, float* ms);

/* Reads and clears the workspace's error flags (workspace NULL: the static
 * scratch of gb_evaluate_static on the plan's device).  Synchronises stream.
 * *flag = 1 if, since the last gb_radii / gb_evaluate call (which clears the
 * flags) or the last check, a fixed-point accumulator would have exceeded 2^62
 * in magnitude (returns GBMC_ERR_OVERFLOW) or a dependency wait of a
 * queued launch gave up (returns GBMC_ERR_HIP; the results of that call
 * are not valid). */
gbmc_status gbmc_check_overflow(const gbmc_plan* plan, void* workspace, hipStream_t stream,
                                int32_t* flag);

#ifdef __cplusplus
}
#endif

#endif /* GBMC_H */
