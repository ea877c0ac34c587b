// Internal declarations shared by the host runtime and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gbmc {

constexpr int kTile = 64;                 // atoms per block; one wavefront per tile
constexpr int kMaxSiteAtoms = 256;
constexpr int kMaxStates = 8;
constexpr int kMaxSweepSites = 1024;      // sites of one kind per system in mc_sweep
constexpr int kMaxSweepSiteAtoms = 1024;  // site atoms per system in mc_sweep (LDS)
#ifndef GBMC_PHI_CHUNK
#define GBMC_PHI_CHUNK 32
#endif
constexpr int kPhiChunk = GBMC_PHI_CHUNK;            // j atoms per FP64 potential-row work item

constexpr double kKB = 1.98720426e-3;      // kcal/(mol K)
constexpr double kFaraday = 23.0605478;    // kcal/(mol V)

// Fixed-point scales (powers of two, so scaling is exact).
constexpr double kScaleI = 4503599627370496.0;   // 2^52: descreening sums, 1/A
constexpr double kScaleF = 1099511627776.0;      // 2^40: forces, dE/dR, dE/dq, dE/drho
constexpr double kScaleE = 4294967296.0;         // 2^32: energies
constexpr double kScaleP = 17592186044416.0;     // 2^44: FP64 site-atom potentials
constexpr double kFixLimit = 4611686018427387904.0;  // 2^62

template <typename T>
struct alignas(4 * sizeof(T)) Q4 {
    T x, y, z, w;
};

// One pair work item: system `sys` (atoms [base, base+n)), the `rows` (1 or 2)
// i blocks [I, I + rows), j blocks [J0, J1) with J0 >= I (J0 >= I + 2 for two
// rows); blk0 is the batch-wide index of the system's first block.
struct WorkItem {
    int32_t base, n, sys, I, J0, J1, rows, blk0;
};

// One 64-atom block of the batch (processing order): atoms [start, start + count).
struct BlockSpan {
    int32_t start, count;
};

// One work item of a cutoff pass, written on the device: i block I of the
// system at [base, base + n) against the j blocks J0 + k, k < J1 - J0 <= 64,
// whose bit k is set in the mask (mask_hi:mask_lo); at most kCutTiles bits.
struct CutItem {
    int32_t base, n, I, J0, J1, blk0;
    uint32_t mask_lo, mask_hi;
};
constexpr int kCutTiles = 4;
constexpr int kCutChunk = 64;            // j blocks per chunk of a block row

// Static tables of the cutoff passes: the 64-atom blocks of the batch and the
// chunks of 64 j blocks of every block row that the compaction kernel scans.
struct CutPlan {
    const BlockSpan* blocks;
    int n_blocks;
    const WorkItem* chunks;
    int n_chunks;
};

// One FP64 potential-row work item: up to 64 site atoms [sa0, sa1) of one system
// against the system's atoms [j0, j1); each lane adds its partial sum in fixed
// point to phi_fx[out + k] (the flattened site-atom slot).
struct RowItem {
    int32_t base, n, sa0, sa1, j0, j1, out, pad;
};

// One atom as the FP64 Monte Carlo kernels read it (caller order; written by
// the radii pass): a 64-byte record, so a wave-uniform read is one scalar
// 64-byte load.
struct alignas(64) Row64 {
    double x, y, z, R, A, pad0, pad1, pad2;   // A = 1 / (2 R)
};

// Device pointers carved from the caller's workspace.  Per-atom arrays marked
// "internal" are in the plan's processing order (perm[k] is the caller index
// of internal atom k); the FP64 per-atom state is in caller order.
template <typename T>
struct Work {
    const int32_t* perm;          // [N] internal -> caller index (plan memory)
    Q4<T>* P;                     // [N] internal: x, y, z, q
    Q4<T>* Gx;                    // [N] internal: rho - offset, screen (rho - offset), screen, 0
    unsigned long long* I_fx;     // [N] internal
    unsigned long long* F_fx;     // [3][N] internal (component-major: one atomic
                                  //  instruction of a wave covers 512 contiguous bytes)
    size_t n_atoms;               // N, the stride of F_fx
    unsigned long long* G_fx;     // [N] internal
    unsigned long long* phi_fx;   // [N] internal
    unsigned long long* drho_fx;  // [N] internal
    unsigned long long* EA_fx;    // [2][N] internal: per-atom Coulomb and GB energy shares
    const int32_t* atom_offset;   // [B+1] (plan memory)
    double* I64;                  // [N] descreening sum
    double* R64;                  // [N] Born radius
    double* A64;                  // [N] 1 / (2 R)
    Row64* rows;                  // [N] FP64 records for the Monte Carlo kernels
    double* T64;                  // [N] tanh(theta)
    double* dRdPsi64;             // [N]
    double* dRdPsi_p;             // [N] internal: dR/dPsi in processing order (the chain
                                  //  pass forms B rt from it and G_fx)
    T* R_t;                       // [N] internal: Born radius in the pair precision
    T* a_t;                       // [N] internal: sqrt(log2(e)/4) / R
    int* ovf;                     // [2]: fixed-point overflow; a wait of a queued
                                  //  launch gave up (both since the last radii call)
    int* qhead;                   // [kQueueWords]: ticket counter ([0]) and error word ([32])
                                  //  of the queued launch
    int* qcnt;                    // [3][n_blocks]: per-block item counters of the passes
    Q4<float>* bnd;               // [n_blocks] bounding sphere of each block: centre, radius
    float* smax;                  // [n_blocks] largest S = screen (rho - offset) of each block
    Q4<float>* box;               // [2][n_blocks] coordinate box of each block (processing
                                  //  order), written by staging: [2b] = lowest x, y, z and
                                  //  largest S, [2b + 1] = highest x, y, z and largest rt
    CutItem* citems[2];           // [cut_cap] each: compacted items (0: descreening and
                                  //  chain passes, 1: energy pass)
    int* ccount;                  // [2] their counts
    int cut_cap;                  // capacity of each list: n_chunks * (kCutChunk / kCutTiles)
};

// What a staging kernel clears besides packing the atoms: up to two runs of
// fixed-point accumulators ([n_acc][N] int64 each), two small int flag arrays
// and an int counter array.
struct StageClear {
    unsigned long long* acc0 = nullptr;
    int n_acc0 = 0;
    unsigned long long* acc1 = nullptr;
    int n_acc1 = 0;
    int* f0 = nullptr;
    int n_f0 = 0;
    int* f1 = nullptr;
    int n_f1 = 0;
    int* cnt = nullptr;
    int n_cnt = 0;
};

struct SiteDev {
    int32_t n_sites, n_cand, n_rowitems;
    int32_t n_site_atoms;             // flattened site-atom slots (site_atom_offset[S])
    const int32_t* site_system;
    const int32_t* site_kind;
    const int32_t* site_atom_offset;
    const int32_t* site_atoms;
    const int32_t* site_state_offset;
    const int32_t* state_charge_offset;
    const double* state_charges;
    const double* state_gref;
    const int32_t* state_count;
    const int32_t* cand_offset;       // [S+1]
    const int32_t* sys_prot_offset;   // [B+1] CSR into sys_prot_sites
    const int32_t* sys_prot_sites;
    const int32_t* sys_redox_offset;  // [B+1]
    const int32_t* sys_redox_sites;
    const int32_t* site_sa_offset;    // [S+1]: first flattened site-atom slot of each site
    const int32_t* sys_sa_offset;     // [B+1]
    const RowItem* rowitems;
};

struct GBConst {
    double alpha, beta, gamma, offset;
    double kC;      // k / eps_in
    double kT;      // k (1/eps_in - 1/eps_out)
    double kO;      // k / eps_out
    double kappa;   // inverse Debye length (1/A); 0: no salt
    double rgbmax;  // descreening cutoff (A); 0: none
    double cutoff;  // pair cutoff of the energy terms (A); 0: none
};

// Energy cutoff in the pair precision: cE = cutoff, cE2 = cutoff^2.
template <typename T>
struct CutK {
    T cE, cE2;
};

// Salt constants of the pair precision: kO = k/eps_out, kap = kappa,
// kap2 = kappa log2(e) (exp(-kappa f) = exp2(-kap2 f)).
template <typename T>
struct SaltK {
    T kO, kap, kap2;
};

// Kernel ids of the timing hook (events ev[2 id] / ev[2 id + 1] bracket a kernel).
// kKRadii, kKEnergy, kKChain: the passes as separate launches (with cutoffs);
// kKRadii also the queued launch of the descreening pass alone, kKForce
// the queued launch of the energy and chain passes, kKEval the queued
// launch of all three.
enum KernelId { kKRadii = 0, kKEnergy = 1, kKChain = 2, kKSiteRows = 3, kKSiteDE = 4, kKMCStep = 5,
                kKForce = 6, kKEval = 7, kNumKernels = 8 };

// Launchers (gbmc_kernels.hip).  All return hipSuccess or the launch error.
// ev (nullable) holds 2 * kNumKernels events: the start and stop events bound to
// the dispatch of each timed kernel.
template <typename T>
hipError_t launch_radii(const WorkItem* items, int n_items, int waves_per_group, int n_atoms,
                        const CutPlan& cp,
                        const T* x, const T* y, const T* z, const T* rho, const T* screen,
                        const GBConst& c, const Work<T>& w, T* born_R, hipStream_t s,
                        hipEvent_t* ev, const T* q = nullptr);
struct PassShape {
    const WorkItem* items;
    int n_items;
    int waves_per_group;
    bool one_tile;          // every item is a single tile (one j block per item)
};

template <typename T>
hipError_t launch_energy_forces(const PassShape& energy, const PassShape& chain, int n_atoms,
                                int n_sys, const CutPlan& cp,
                                const T* x, const T* y, const T* z, const T* q, const T* rho,
                                const T* screen, const GBConst& c, const Work<T>& w,
                                double* e_coul, double* e_gb, T* force, T* dEdq, T* dEdrho,
                                hipStream_t s, hipEvent_t* ev, bool staged = false);
// Ints of the workspace taken by the queued launch's ticket counter and error
// word (on separate 128-byte lines).
constexpr int kQueueWords = 64;

// The queued launch of the all-pairs passes: the plan's three work
// lists, the number of items of each pass touching each 64-atom block
// ([3][n_blocks], plan memory) and the launch parameters.
struct QueueShape {
    const WorkItem* items[3];
    int n_items[3];
    const int* total;
    const BlockSpan* blocks;  // [n_blocks] atoms of each block (processing order)
    int n_blocks;
    bool one_tile;          // energy and chain items are single tiles
    int spin_limit;         // polls before a dependency wait gives up
    int n_cu;               // compute units of the device
};

// Staging, the three all-pairs passes (descreening, energy / explicit
// forces with gradients, Born chain) in one queued launch, and the outputs.
template <typename T>
hipError_t launch_queued(const QueueShape& sh, int n_atoms, int n_sys, const T* x, const T* y,
                         const T* z, const T* q, const T* rho, const T* screen, const GBConst& c,
                         const Work<T>& w, T* born_R, double* e_coul, double* e_gb, T* force,
                         T* dEdq, T* dEdrho, hipStream_t s, hipEvent_t* ev, int timing_id);

template <typename T>
hipError_t launch_state_dE(const SiteDev& sd, int n_atoms, const T* x, const T* y, const T* z,
                           const T* q, const GBConst& c, const Work<T>& w, unsigned long long* phi_fx,
                           const int32_t* current_state, const double* pH, const double* E_volt,
                           double T_kelvin, double* dE, double* dG, hipStream_t s,
                           hipEvent_t* ev);
template <typename T>
hipError_t launch_mc_step(const SiteDev& sd, int n_sys, const T* x, const T* y, const T* z,
                          T* q, const GBConst& c, const Work<T>& w, int32_t* current_state,
                          const double* pH, const double* E_volt, double T_kelvin,
                          const double* dE, const double* dG, const double* u,
                          int32_t* n_electrons, int64_t* counters, int32_t* accepted,
                          hipStream_t s, hipEvent_t* ev);
template <typename T>
hipError_t launch_mc_sweep(const SiteDev& sd, int n_sys, int n_sa_max, const T* x, const T* y,
                           const T* z, const T* q, T* q_out, const GBConst& c, const Work<T>& w,
                           unsigned long long* phi_fx, int32_t* current_state, const double* pH,
                           const double* E_volt, double T_kelvin, int kinds, const double* u,
                           int32_t* n_electrons, int64_t* counters, int32_t* accepted, double* dG,
                           hipStream_t s);
template <typename T>
hipError_t launch_md_langevin(int n, T* x, T* y, T* z, T* v, const T* force, const T* inv_mass,
                              const T* xi, const T* xref, double k_restr, double dt, double gamma,
                              double T_kelvin, hipStream_t s);
size_t plain_workspace_bytes(int n_atoms);
hipError_t launch_plain_fp64(int n_sys, const int32_t* atom_offset, int n_atoms, const double* x,
                             const double* y, const double* z, const double* q, const double* rho,
                             const double* screen, const GBConst& c, void* workspace,
                             double* born_R, double* e_coul, double* e_gb, double* force,
                             double* dEdq, double* dEdrho, hipStream_t s);
// Library-owned device scratch of gb_evaluate_static (one per GPU): its size
// and its device address on `device`, which must be the current device
// (resolved with hipGetSymbolAddress on the first request per device).
constexpr size_t kScratchBytes = (size_t)256 << 20;
hipError_t scratch_address(int device, void** ptr);

hipError_t launch_remd_exchange(int M, const double* E_rung, const int32_t* Ne, int32_t* rep,
                                double T_kelvin, int parity, int wrap, const double* u,
                                int32_t* accepted, double* E_of_rep, hipStream_t s);

}  // namespace gbmc
