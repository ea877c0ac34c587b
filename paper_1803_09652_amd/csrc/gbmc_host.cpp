// gbmc_host.cpp -- host runtime behind the C ABI in include/gbmc.h: plans,
// work schedules, validation, workspace layout and kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <exception>
#include <initializer_list>
#include <new>
#include <utility>
#include <string>
#include <vector>

#include "gbmc.h"
#include "gbmc_internal.h"

using namespace gbmc;

namespace {

thread_local std::string g_last_error;

gbmc_status fail(gbmc_status st, const std::string& msg)
{
    g_last_error = msg;
    return st;
}

gbmc_status hip_fail(hipError_t e, const char* where)
{
    return fail(GBMC_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

constexpr int64_t kTimedMax = 256;   // launches kept per timed kernel between reads

// Default work shapes (radii, energy, chain): one 64-atom j block per work
// item in every pass (single-tile items, the instantiations with the fewest
// registers), with the waves per workgroup measured fastest on batches of tens
// of thousands of atoms.  FP32 batches of at least kLongItemTiles tiles (which
// fill the GPU many times over even in items of four tiles) take four j
// blocks per item and one wave per workgroup in the energy and chain passes:
// fewer i-side flushes and per-item loads, measured 2-4 % faster on a batch of
// 64 systems of 1,000-20,000 atoms (and 40-50 % slower on 16 systems of 2,500).
const gbmc_tuning kDefaultTuning32 = {{1, 1, 1}, {2, 4, 4}};
const gbmc_tuning kDefaultTuning64 = {{1, 1, 1}, {2, 2, 2}};
constexpr int64_t kLongItemTiles = int64_t(1) << 19;

// Queued launch: the polls (each after a short sleep, about a microsecond
// apiece) before a dependency wait gives up: seconds, far beyond any wait the
// schedule produces.
constexpr int kDefaultSpinLimit = 1 << 22;

}  // namespace

struct gbmc_plan {
    int32_t n_sys = 0;
    int32_t n_atoms = 0;
    gbmc_precision prec = GBMC_FP32_FIXED;
    gbmc_tuning tuning = kDefaultTuning32;
    std::vector<int32_t> offset;     // [B+1]
    int32_t n_items[GBMC_N_PASSES] = {0, 0, 0};
    WorkItem* d_items[GBMC_N_PASSES] = {nullptr, nullptr, nullptr};
    void* d_mem = nullptr;           // one allocation: the work lists and the order
    int32_t* d_perm = nullptr;       // [N] internal -> caller atom index
    int32_t* d_offset = nullptr;     // [B+1] device copy of the atom offsets
    int32_t n_blocks = 0;            // 64-atom blocks of the batch
    BlockSpan* d_blocks = nullptr;   // [n_blocks] atoms of each block (processing order)
    int32_t* d_total = nullptr;      // [3][n_blocks] items of each pass touching each block
    int n_cu = 0;                    // compute units of the device
    bool single_launch = false;           // gb_evaluate as one queued launch
    int spin_limit = kDefaultSpinLimit;   // polls before a wait of a queued launch gives up
    int32_t n_chunks = 0;            // cutoff passes: block rows in chunks of 64 j blocks
    WorkItem* d_chunks = nullptr;
    int device = 0;
    void* scratch = nullptr;         // the library's static scratch on `device`
    hipError_t scratch_err = hipSuccess;
    hipEvent_t fork_ev = nullptr;    // gb_evaluate_fork: recorded when the radii are final
    // timing hook: a ring of start/stop event pairs per timed kernel (bound to
    // the dispatches while enabled), the launches recorded since the last
    // read, and the pairs handed to the current call
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;  // [kNumKernels][kTimedMax][2]
    int64_t n_rec[kNumKernels] = {};
    hipEvent_t cur[2 * kNumKernels] = {};
    // workspace layout (byte offsets)
    size_t off_I, off_F, off_G, off_phi, off_drho, off_EA, off_I64, off_R64, off_T64, off_dR64, off_dRp,
        off_Rt, off_at, off_ovf, off_q, off_P, off_Gx, off_A64, off_rows, off_bnd,
        off_smax, off_box, off_cit0, off_cit1, off_ccount, ws_bytes;
    int32_t cut_cap = 0;             // capacity of each compacted cutoff work list
};

struct gbmc_sites {
    const gbmc_plan* plan = nullptr;
    int32_t n_sites = 0, n_cand = 0, n_rowitems = 0;
    size_t n_site_atoms = 0;         // fixed-point potential slots in the site workspace
    int32_t max_sys_site_atoms = 0;  // largest number of site atoms in one system
    int32_t max_sys_sites = 0;       // largest number of sites of one kind in one system
    void* d_mem = nullptr;
    SiteDev dev{};
};

// ------------------------------------------------------------------ schedule

static gbmc_status check_offsets(int32_t n_systems, const int32_t* off)
{
    if (n_systems < 0) return fail(GBMC_ERR_INVALID, "n_systems < 0");
    if (n_systems > 0 && !off) return fail(GBMC_ERR_INVALID, "atom_offset is NULL");
    if (n_systems == 0) return GBMC_OK;
    if (off[0] != 0) return fail(GBMC_ERR_INVALID, "atom_offset[0] must be 0");
    for (int32_t b = 0; b < n_systems; ++b) {
        if (off[b + 1] < off[b]) return fail(GBMC_ERR_INVALID, "atom_offset must be non-decreasing");
        if ((int64_t)off[b + 1] - off[b] > (int64_t)kTile * 65535)
            return fail(GBMC_ERR_UNSUPPORTED, "a system has more than 4,194,240 atoms");
    }
    return GBMC_OK;
}

// With row_pairs, the i blocks of a system are taken in pairs (2a, 2a + 1):
// the tiles of the pair against j blocks J >= 2a + 2 form two-row items; the
// diagonal band (2a, 2a), (2a, 2a + 1), (2a + 1, 2a + 1) and an unpaired last
// block form one-row items.  Without, every i block has one-row items.  Each
// run of j blocks is cut into items of at most jb blocks.
static gbmc_status build_items(int32_t n_systems, const int32_t* off, int32_t jb, bool row_pairs,
                               std::vector<WorkItem>& items)
{
    items.clear();
    int32_t blk0 = 0;
    auto add = [&](int32_t b, int32_t rows, int32_t I, int32_t J0, int32_t J1) {
        for (int32_t j = J0; j < J1; j += jb) {
            WorkItem w{};
            w.base = off[b];
            w.n = off[b + 1] - off[b];
            w.sys = b;
            w.I = I;
            w.J0 = j;
            w.J1 = std::min(J1, j + jb);
            w.rows = rows;
            w.blk0 = blk0;
            items.push_back(w);
        }
    };
    for (int32_t b = 0; b < n_systems; ++b, blk0 += (off[b] - off[b - 1] + kTile - 1) / kTile) {
        const int32_t nb = (off[b + 1] - off[b] + kTile - 1) / kTile;
        if (!row_pairs) {
            for (int32_t I = 0; I < nb; ++I) add(b, 1, I, I, nb);
            continue;
        }
        for (int32_t a = 0; a < nb; a += 2) {
            if (a + 1 < nb) {
                add(b, 1, a, a, a + 2);
                add(b, 1, a + 1, a + 1, a + 2);
                add(b, 2, a, a + 2, nb);
            } else {
                add(b, 1, a, a, a + 1);
            }
        }
    }
    // longest first (in half tiles: a diagonal tile costs half an off-diagonal
    // one); ties keep the construction order so the schedule is deterministic
    auto cost = [](const WorkItem& w) {
        return 2 * w.rows * (w.J1 - w.J0) - (w.J0 == w.I ? 1 : 0);
    };
    std::stable_sort(items.begin(), items.end(),
                     [&](const WorkItem& a, const WorkItem& b) { return cost(a) > cost(b); });
    return GBMC_OK;
}

// Distinct 64-atom blocks of a work item: its i blocks [I, I + rows), then
// its j blocks [J0, J1) other than those (J0 >= I).  The queued launch
// counts an item done on each of them.
static int32_t item_blocks(const WorkItem& w)
{
    return w.rows + std::max(0, w.J1 - std::max(w.J0, w.I + w.rows));
}
static int32_t item_block(const WorkItem& w, int32_t k)
{
    return k < w.rows ? w.I + k : std::max(w.J0, w.I + w.rows) + (k - w.rows);
}

// The caller's work shapes, checked, or (tuning NULL) the defaults for a batch
// with these offsets.
static gbmc_status check_tuning(const gbmc_tuning* in, gbmc_precision prec, int32_t n_systems,
                                const int32_t* off, gbmc_tuning& out)
{
    out = prec == GBMC_FP64 ? kDefaultTuning64 : kDefaultTuning32;
    if (!in) {
        int64_t tiles = 0;
        for (int32_t b = 0; b < n_systems; ++b) {
            const int64_t nb = (off[b + 1] - off[b] + kTile - 1) / kTile;
            tiles += nb * (nb + 1) / 2;
        }
        if (prec == GBMC_FP32_FIXED && tiles >= kLongItemTiles)
            for (int k : {GBMC_PASS_ENERGY, GBMC_PASS_CHAIN}) {
                out.j_blocks_per_item[k] = 4;
                out.waves_per_group[k] = 1;
            }
        return GBMC_OK;
    }
    for (int k = 0; k < GBMC_N_PASSES; ++k) {
        if (in->j_blocks_per_item[k] < 1 || in->j_blocks_per_item[k] > 65535)
            return fail(GBMC_ERR_INVALID, "tuning.j_blocks_per_item must be in [1, 65535]");
        const int32_t wv = in->waves_per_group[k];
        if (wv != 1 && wv != 2 && wv != 4 && wv != 8)
            return fail(GBMC_ERR_INVALID, "tuning.waves_per_group must be 1, 2, 4 or 8");
    }
    out = *in;
    return GBMC_OK;
}

template <typename T>
static Work<T> carve(const gbmc_plan* p, void* ws)
{
    char* b = static_cast<char*>(ws);
    Work<T> w;
    w.perm = p->d_perm;
    w.atom_offset = p->d_offset;
    w.P = reinterpret_cast<Q4<T>*>(b + p->off_P);
    w.Gx = reinterpret_cast<Q4<T>*>(b + p->off_Gx);
    w.I_fx = reinterpret_cast<unsigned long long*>(b + p->off_I);
    w.F_fx = reinterpret_cast<unsigned long long*>(b + p->off_F);
    w.n_atoms = (size_t)p->n_atoms;
    w.G_fx = reinterpret_cast<unsigned long long*>(b + p->off_G);
    w.phi_fx = reinterpret_cast<unsigned long long*>(b + p->off_phi);
    w.drho_fx = reinterpret_cast<unsigned long long*>(b + p->off_drho);
    w.EA_fx = reinterpret_cast<unsigned long long*>(b + p->off_EA);
    w.I64 = reinterpret_cast<double*>(b + p->off_I64);
    w.R64 = reinterpret_cast<double*>(b + p->off_R64);
    w.A64 = reinterpret_cast<double*>(b + p->off_A64);
    w.rows = reinterpret_cast<Row64*>(b + p->off_rows);
    w.T64 = reinterpret_cast<double*>(b + p->off_T64);
    w.dRdPsi64 = reinterpret_cast<double*>(b + p->off_dR64);
    w.dRdPsi_p = reinterpret_cast<double*>(b + p->off_dRp);
    w.R_t = reinterpret_cast<T*>(b + p->off_Rt);
    w.a_t = reinterpret_cast<T*>(b + p->off_at);
    w.ovf = reinterpret_cast<int*>(b + p->off_ovf);
    w.qhead = reinterpret_cast<int*>(b + p->off_q);
    w.qcnt = reinterpret_cast<int*>(b + p->off_q + 4 * (size_t)kQueueWords);
    w.bnd = reinterpret_cast<Q4<float>*>(b + p->off_bnd);
    w.smax = reinterpret_cast<float*>(b + p->off_smax);
    w.box = reinterpret_cast<Q4<float>*>(b + p->off_box);
    w.citems[0] = reinterpret_cast<CutItem*>(b + p->off_cit0);
    w.citems[1] = reinterpret_cast<CutItem*>(b + p->off_cit1);
    w.ccount = reinterpret_cast<int*>(b + p->off_ccount);
    w.cut_cap = p->cut_cap;
    return w;
}

static void layout(gbmc_plan* p)
{
    const size_t N = (size_t)p->n_atoms, B = (size_t)p->n_sys;
    const size_t ts = p->prec == GBMC_FP64 ? 8 : 4;
    size_t o = 0;
    auto seg = [&](size_t bytes) { size_t at = o; o = align256(o + bytes); return at; };
    p->off_I = seg(8 * (N + 1));           // the overflow word follows I_fx
    p->off_ovf = p->off_I + 8 * N;
    // F (3N), G, phi, drho and the energy shares (2N) are one contiguous run of
    // 8N int64: cleared by one kernel
    p->off_F = seg(8 * 8 * N);
    p->off_G = p->off_F + 8 * 3 * N;
    p->off_phi = p->off_G + 8 * N;
    p->off_drho = p->off_phi + 8 * N;
    p->off_EA = p->off_drho + 8 * N;
    (void)B;
    p->off_I64 = seg(8 * N);
    p->off_R64 = seg(8 * N);
    p->off_A64 = seg(8 * N);
    p->off_T64 = seg(8 * N);
    p->off_dR64 = seg(8 * N);
    p->off_dRp = seg(8 * N);
    p->off_Rt = seg(ts * N);
    p->off_at = seg(ts * N);
    p->off_P = seg(4 * ts * N);
    p->off_Gx = seg(4 * ts * N);
    p->off_rows = seg(sizeof(Row64) * N);
    p->off_bnd = seg(sizeof(Q4<float>) * (size_t)p->n_blocks);
    p->off_smax = seg(sizeof(float) * (size_t)p->n_blocks);
    p->off_box = seg(2 * sizeof(Q4<float>) * (size_t)p->n_blocks);
    p->off_cit0 = seg(sizeof(CutItem) * (size_t)p->cut_cap);
    p->off_cit1 = seg(sizeof(CutItem) * (size_t)p->cut_cap);
    p->off_ccount = seg(2 * sizeof(int));
    // queue counters (one 128-byte line each), the error word, block counters
    p->off_q = seg(4 * (size_t)kQueueWords + 4 * 3 * (size_t)p->n_blocks);
    p->ws_bytes = o;
}

static CutPlan cut_plan(const gbmc_plan* p)
{
    return CutPlan{p->d_blocks, p->n_blocks, p->d_chunks, p->n_chunks};
}

static GBConst make_const(const gbmc_gb_params* gp)
{
    GBConst c;
    c.alpha = gp->alpha;
    c.beta = gp->beta;
    c.gamma = gp->gamma;
    c.offset = gp->offset;
    c.kC = gp->coulomb_k / gp->eps_in;
    c.kT = gp->coulomb_k * (1.0 / gp->eps_in - 1.0 / gp->eps_out);
    c.kO = gp->coulomb_k / gp->eps_out;
    c.kappa = gp->kappa;
    c.rgbmax = gp->rgbmax;
    c.cutoff = gp->cutoff;
    return c;
}

static gbmc_status check_call(const gbmc_plan* p, const gbmc_atoms* a, const gbmc_gb_params* gp,
                              const void* ws, bool need_q)
{
    if (!p) return fail(GBMC_ERR_INVALID, "plan is NULL");
    if (!gp) return fail(GBMC_ERR_INVALID, "params is NULL");
    gbmc_status st = gbmc_params_validate(gp);
    if (st != GBMC_OK) return st;
    if (p->n_atoms == 0) return GBMC_OK;
    if (!a || !a->x || !a->y || !a->z || !a->rho || !a->screen || (need_q && !a->q))
        return fail(GBMC_ERR_INVALID, "an atom array is NULL");
    if (!ws) return fail(GBMC_ERR_INVALID, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0)
        return fail(GBMC_ERR_INVALID, "workspace must be 256-byte aligned");
    return GBMC_OK;
}

// ------------------------------------------------------------------ C ABI

extern "C" {

int32_t gbmc_version(void) { return 10000; }

const char* gbmc_last_error(void) { return g_last_error.c_str(); }

gbmc_status gbmc_params_validate(const gbmc_gb_params* p)
{
    if (!p) return fail(GBMC_ERR_INVALID, "params is NULL");
    const double v[] = {p->alpha, p->beta, p->gamma, p->offset, p->eps_in, p->eps_out,
                        p->coulomb_k, p->kappa, p->rgbmax, p->cutoff};
    for (double x : v)
        if (!std::isfinite(x)) return fail(GBMC_ERR_INVALID, "non-finite GB parameter");
    if (p->kappa < 0.0) return fail(GBMC_ERR_INVALID, "kappa must be >= 0");
    if (p->rgbmax < 0.0 || p->cutoff < 0.0) return fail(GBMC_ERR_INVALID, "cutoffs must be >= 0 (0: none)");
    if (p->eps_in <= 0.0 || p->eps_out <= 0.0) return fail(GBMC_ERR_INVALID, "dielectric constants must be > 0");
    if (p->offset < 0.0) return fail(GBMC_ERR_INVALID, "offset must be >= 0");
    return GBMC_OK;
}

// The work lists of a plan, one per pass (build_items with the pass's j
// blocks per item; two-row items in the energy and chain passes of FP32
// plans), and the
// number of items of each pass touching each 64-atom block (the counts the
// queued launch's per-block counters complete at).  The queued launch runs a
// pass's items before the next pass's, and a block of the next pass can start
// once every item touching it is done, so the descreening and energy passes
// take their items system by system (largest system first, each system's
// items by decreasing cost): whole systems finish early and the next pass
// starts on them while the last systems finish.  The chain pass, which ends
// the launch, keeps the global decreasing-cost order.
static void plan_schedule(int32_t n_systems, const int32_t* off, gbmc_precision prec,
                          const gbmc_tuning& t, std::vector<WorkItem> (&items)[GBMC_N_PASSES],
                          int32_t& n_blocks, std::vector<int32_t>& totals)
{
    for (int k = 0; k < GBMC_N_PASSES; ++k)
        build_items(n_systems, off, t.j_blocks_per_item[k],
                    prec == GBMC_FP32_FIXED && k != GBMC_PASS_RADII, items[k]);
    std::vector<int32_t> rank(n_systems);
    for (int32_t b = 0; b < n_systems; ++b) rank[b] = b;
    std::stable_sort(rank.begin(), rank.end(), [&](int32_t a, int32_t c) {
        return off[a + 1] - off[a] > off[c + 1] - off[c];
    });
    std::vector<int32_t> pos(n_systems);
    for (int32_t r = 0; r < n_systems; ++r) pos[rank[r]] = r;
    for (int k : {GBMC_PASS_RADII, GBMC_PASS_ENERGY})
        std::stable_sort(items[k].begin(), items[k].end(),
                         [&](const WorkItem& a, const WorkItem& c) { return pos[a.sys] < pos[c.sys]; });
    n_blocks = 0;
    for (int32_t b = 0; b < n_systems; ++b) n_blocks += (off[b + 1] - off[b] + kTile - 1) / kTile;
    totals.assign((size_t)GBMC_N_PASSES * n_blocks, 0);
    for (int k = 0; k < GBMC_N_PASSES; ++k)
        for (const WorkItem& w : items[k])
            for (int32_t d = 0; d < item_blocks(w); ++d)
                ++totals[(size_t)k * n_blocks + w.blk0 + item_block(w, d)];
}

gbmc_status gbmc_schedule_build(int32_t n_systems, const int32_t* host_atom_offset,
                                int32_t j_blocks_per_item, int32_t row_pairs, int32_t* n_items,
                                int32_t* items)
{
    try {
        if (!n_items) return fail(GBMC_ERR_INVALID, "n_items is NULL");
        gbmc_status st = check_offsets(n_systems, host_atom_offset);
        if (st != GBMC_OK) return st;
        if (j_blocks_per_item < 1 || j_blocks_per_item > 65535)
            return fail(GBMC_ERR_INVALID, "j_blocks_per_item must be in [1, 65535]");
        std::vector<WorkItem> v;
        build_items(n_systems, host_atom_offset, j_blocks_per_item, row_pairs != 0, v);
        if (v.size() > 0x7fffffff) return fail(GBMC_ERR_UNSUPPORTED, "too many work items");
        *n_items = (int32_t)v.size();
        if (items)
            for (size_t k = 0; k < v.size(); ++k) {
                items[5 * k + 0] = v[k].sys;
                items[5 * k + 1] = v[k].I;
                items[5 * k + 2] = v[k].I + v[k].rows;
                items[5 * k + 3] = v[k].J0;
                items[5 * k + 4] = v[k].J1;
            }
        return GBMC_OK;
    } catch (const std::exception& e) {
        return fail(GBMC_ERR_INVALID, e.what());
    }
}

gbmc_status gbmc_queue_schedule(int32_t n_systems, const int32_t* host_atom_offset,
                                gbmc_precision precision, const gbmc_tuning* tuning,
                                int32_t* n_items, int32_t* items, int32_t* n_blocks,
                                int32_t* totals)
{
    try {
        if (!n_items || !n_blocks) return fail(GBMC_ERR_INVALID, "n_items or n_blocks is NULL");
        gbmc_status st = check_offsets(n_systems, host_atom_offset);
        if (st != GBMC_OK) return st;
        if (precision != GBMC_FP32_FIXED && precision != GBMC_FP64)
            return fail(GBMC_ERR_INVALID, "unknown precision");
        gbmc_tuning t;
        st = check_tuning(tuning, precision, n_systems, host_atom_offset, t);
        if (st != GBMC_OK) return st;
        std::vector<WorkItem> v[GBMC_N_PASSES];
        std::vector<int32_t> tot;
        int32_t nb = 0;
        plan_schedule(n_systems, host_atom_offset, precision, t, v, nb, tot);
        size_t all = 0;
        for (int k = 0; k < GBMC_N_PASSES; ++k) all += v[k].size();
        if (all > 0x7fffffff / 7) return fail(GBMC_ERR_UNSUPPORTED, "too many work items");
        for (int k = 0; k < GBMC_N_PASSES; ++k) n_items[k] = (int32_t)v[k].size();
        *n_blocks = nb;
        if (items) {
            size_t r = 0;
            for (int k = 0; k < GBMC_N_PASSES; ++k)
                for (const WorkItem& w : v[k]) {
                    int32_t* o = items + 7 * r++;
                    o[0] = k;
                    o[1] = w.sys;
                    o[2] = w.blk0;
                    o[3] = w.I;
                    o[4] = w.I + w.rows;
                    o[5] = w.J0;
                    o[6] = w.J1;
                }
        }
        if (totals && !tot.empty()) std::memcpy(totals, tot.data(), sizeof(int32_t) * tot.size());
        return GBMC_OK;
    } catch (const std::bad_alloc&) {
        return fail(GBMC_ERR_INVALID, "host allocation failed");
    }
}

gbmc_status gbmc_plan_create(gbmc_plan** out, int32_t n_systems, const int32_t* host_atom_offset,
                             gbmc_precision precision, const gbmc_tuning* tuning)
{
    try {
        if (!out) return fail(GBMC_ERR_INVALID, "plan out-pointer is NULL");
        *out = nullptr;
        gbmc_status st = check_offsets(n_systems, host_atom_offset);
        if (st != GBMC_OK) return st;
        if (precision != GBMC_FP32_FIXED && precision != GBMC_FP64)
            return fail(GBMC_ERR_INVALID, "unknown precision");
        gbmc_tuning t;
        st = check_tuning(tuning, precision, n_systems, host_atom_offset, t);
        if (st != GBMC_OK) return st;
        std::vector<WorkItem> items[GBMC_N_PASSES];
        std::vector<int32_t> totals;
        int32_t n_blocks = 0;
        plan_schedule(n_systems, host_atom_offset, precision, t, items, n_blocks, totals);
        auto* p = new gbmc_plan();
        p->n_sys = n_systems;
        p->n_atoms = n_systems > 0 ? host_atom_offset[n_systems] : 0;
        p->prec = precision;
        p->tuning = t;
        p->offset.assign(host_atom_offset, host_atom_offset + n_systems + 1);
        if (n_systems == 0) p->offset.assign(1, 0);
        std::vector<BlockSpan> blocks;
        for (int32_t b = 0; b < n_systems; ++b)
            for (int32_t a = host_atom_offset[b]; a < host_atom_offset[b + 1]; a += kTile)
                blocks.push_back(BlockSpan{a, std::min(kTile, host_atom_offset[b + 1] - a)});
        p->n_blocks = (int32_t)blocks.size();
        if (p->n_blocks != n_blocks) {
            delete p;
            return fail(GBMC_ERR_INVALID, "internal: block count mismatch");
        }
        // chunks of the cutoff passes: every block row against its j blocks,
        // 64 at a time (the compaction kernel scans one chunk per wave)
        std::vector<WorkItem> chunks;
        build_items(n_systems, host_atom_offset, kCutChunk, false, chunks);
        if ((uint64_t)chunks.size() * (kCutChunk / kCutTiles) > 0x7fffffffull) {
            delete p;
            return fail(GBMC_ERR_UNSUPPORTED, "too many blocks for the cutoff work lists");
        }
        p->n_chunks = (int32_t)chunks.size();
        p->cut_cap = p->n_chunks * (kCutChunk / kCutTiles);
        layout(p);
        hipError_t e = hipGetDevice(&p->device);
        if (e != hipSuccess) { delete p; return hip_fail(e, "hipGetDevice"); }
        // the device address of the static scratch of gb_evaluate_static on this
        // device (resolved once per device; a failure only disables that call)
        p->scratch_err = scratch_address(p->device, &p->scratch);
        e = hipDeviceGetAttribute(&p->n_cu, hipDeviceAttributeMultiprocessorCount, p->device);
        if (e != hipSuccess) { delete p; return hip_fail(e, "hipDeviceGetAttribute"); }
        // one device allocation: the three work lists, then the processing order (identity)
        size_t at[GBMC_N_PASSES + 1];
        size_t o = 0;
        for (int k = 0; k < GBMC_N_PASSES; ++k) {
            if (items[k].size() > 0x7fffffff) { delete p; return fail(GBMC_ERR_UNSUPPORTED, "too many work items"); }
            p->n_items[k] = (int32_t)items[k].size();
            at[k] = o;
            o = align256(o + items[k].size() * sizeof(WorkItem));
        }
        at[GBMC_N_PASSES] = o;
        const size_t off_bytes = 4 * (size_t)(n_systems + 1);
        const size_t at_off = align256(o + 4 * (size_t)p->n_atoms);
        const size_t at_blk = align256(at_off + off_bytes);
        const size_t at_chk = align256(at_blk + sizeof(BlockSpan) * blocks.size());
        const size_t at_tot = align256(at_chk + sizeof(WorkItem) * chunks.size());
        const size_t total = at_tot + sizeof(int32_t) * totals.size();
        if (total > 0) {
            char* d = nullptr;
            e = hipMalloc(&d, total);
            if (e != hipSuccess) { delete p; return hip_fail(e, "hipMalloc(plan tables)"); }
            p->d_mem = d;
            std::vector<char> h(total, 0);
            for (int k = 0; k < GBMC_N_PASSES; ++k) {
                p->d_items[k] = reinterpret_cast<WorkItem*>(d + at[k]);
                if (!items[k].empty())
                    std::memcpy(h.data() + at[k], items[k].data(), items[k].size() * sizeof(WorkItem));
            }
            p->d_perm = reinterpret_cast<int32_t*>(d + at[GBMC_N_PASSES]);
            int32_t* id = reinterpret_cast<int32_t*>(h.data() + at[GBMC_N_PASSES]);
            for (int32_t k = 0; k < p->n_atoms; ++k) id[k] = k;
            p->d_offset = reinterpret_cast<int32_t*>(d + at_off);
            std::memcpy(h.data() + at_off, p->offset.data(), off_bytes);
            p->d_blocks = reinterpret_cast<BlockSpan*>(d + at_blk);
            if (!blocks.empty())
                std::memcpy(h.data() + at_blk, blocks.data(), sizeof(BlockSpan) * blocks.size());
            p->d_chunks = reinterpret_cast<WorkItem*>(d + at_chk);
            if (!chunks.empty())
                std::memcpy(h.data() + at_chk, chunks.data(), sizeof(WorkItem) * chunks.size());
            p->d_total = reinterpret_cast<int32_t*>(d + at_tot);
            if (!totals.empty())
                std::memcpy(h.data() + at_tot, totals.data(), sizeof(int32_t) * totals.size());
            e = hipMemcpy(d, h.data(), h.size(), hipMemcpyHostToDevice);
            if (e != hipSuccess) { (void)hipFree(d); delete p; return hip_fail(e, "hipMemcpy(plan tables)"); }
        }
        e = hipEventCreateWithFlags(&p->fork_ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            if (p->d_mem) (void)hipFree(p->d_mem);
            delete p;
            return hip_fail(e, "hipEventCreateWithFlags");
        }
        *out = p;
        return GBMC_OK;
    } catch (const std::bad_alloc&) {
        return fail(GBMC_ERR_INVALID, "host allocation failed");
    }
}

void gbmc_plan_destroy(gbmc_plan* p)
{
    if (!p) return;
    if (p->d_mem) (void)hipFree(p->d_mem);
    for (hipEvent_t e : p->ev_pool)
        if (e) (void)hipEventDestroy(e);
    if (p->fork_ev) (void)hipEventDestroy(p->fork_ev);
    delete p;
}

gbmc_status gbmc_plan_set_timing(gbmc_plan* p, int32_t enable)
{
    if (!p) return fail(GBMC_ERR_INVALID, "plan is NULL");
    if (enable && p->ev_pool.empty()) {
        try {
            p->ev_pool.assign((size_t)2 * kNumKernels * kTimedMax, nullptr);
        } catch (const std::bad_alloc&) {
            return fail(GBMC_ERR_INVALID, "host allocation failed");
        }
        for (hipEvent_t& e : p->ev_pool) {
            hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) return hip_fail(r, "hipEventCreate");
        }
    }
    p->timing = enable != 0;
    for (int64_t& n : p->n_rec) n = 0;
    return GBMC_OK;
}

static hipEvent_t* pool_pair(gbmc_plan* p, int k, int64_t launch)
{
    return &p->ev_pool[2 * ((size_t)k * kTimedMax + (size_t)(launch % kTimedMax))];
}

gbmc_status gbmc_plan_kernel_ms(gbmc_plan* p, float* ms)
{
    if (!p || !ms) return fail(GBMC_ERR_INVALID, "NULL argument");
    for (int k = 0; k < kNumKernels; ++k) {
        ms[k] = -1.0f;
        const int64_t n = p->n_rec[k];
        if (n == 0) continue;
        hipError_t r = hipEventSynchronize(pool_pair(p, k, n - 1)[1]);
        if (r != hipSuccess) return hip_fail(r, "hipEventSynchronize");
        const int64_t m = n < kTimedMax ? n : kTimedMax;   // the most recent launches kept
        double sum = 0.0;
        for (int64_t l = n - m; l < n; ++l) {
            hipEvent_t* e = pool_pair(p, k, l);
            float t = 0.0f;
            r = hipEventElapsedTime(&t, e[0], e[1]);
            if (r != hipSuccess) return hip_fail(r, "hipEventElapsedTime");
            sum += t;
        }
        ms[k] = (float)(sum / (double)m);
        p->n_rec[k] = 0;
    }
    return GBMC_OK;
}

size_t gbmc_plan_workspace_bytes(const gbmc_plan* p) { return p ? p->ws_bytes : 0; }

static gbmc_status check_order(int32_t n_systems, const int32_t* off, const int32_t* order)
{
    const int32_t N = n_systems > 0 ? off[n_systems] : 0;
    if (N > 0 && !order) return fail(GBMC_ERR_INVALID, "order is NULL");
    std::vector<char> seen(N, 0);
    for (int32_t b = 0; b < n_systems; ++b)
        for (int32_t k = off[b]; k < off[b + 1]; ++k) {
            const int32_t c = order[k];
            if (c < off[b] || c >= off[b + 1])
                return fail(GBMC_ERR_INVALID, "order maps an atom outside its system");
            if (seen[c]) return fail(GBMC_ERR_INVALID, "order is not a permutation");
            seen[c] = 1;
        }
    return GBMC_OK;
}

gbmc_status gbmc_plan_set_order(gbmc_plan* p, const int32_t* order)
{
    try {
        if (!p) return fail(GBMC_ERR_INVALID, "plan is NULL");
        gbmc_status st = check_order(p->n_sys, p->offset.data(), order);
        if (st != GBMC_OK) return st;
        if (p->n_atoms == 0) return GBMC_OK;
        hipError_t e = hipMemcpy(p->d_perm, order, 4 * (size_t)p->n_atoms, hipMemcpyHostToDevice);
        return e == hipSuccess ? GBMC_OK : hip_fail(e, "hipMemcpy(order)");
    } catch (const std::bad_alloc&) {
        return fail(GBMC_ERR_INVALID, "host allocation failed");
    }
}

gbmc_status gbmc_spatial_order(int32_t n_systems, const int32_t* off, const double* x,
                               const double* y, const double* z, int32_t* order)
{
    try {
        gbmc_status st = check_offsets(n_systems, off);
        if (st != GBMC_OK) return st;
        const int32_t N = n_systems > 0 ? off[n_systems] : 0;
        if (N > 0 && (!x || !y || !z || !order)) return fail(GBMC_ERR_INVALID, "NULL argument");
        std::vector<std::pair<uint64_t, int32_t>> key;
        for (int32_t b = 0; b < n_systems; ++b) {
            const int32_t a0 = off[b], a1 = off[b + 1];
            if (a1 == a0) continue;
            double lo[3] = {x[a0], y[a0], z[a0]}, hi[3] = {x[a0], y[a0], z[a0]};
            for (int32_t k = a0; k < a1; ++k) {
                const double v[3] = {x[k], y[k], z[k]};
                for (int d = 0; d < 3; ++d) {
                    if (!std::isfinite(v[d])) return fail(GBMC_ERR_INVALID, "non-finite coordinate");
                    lo[d] = std::min(lo[d], v[d]);
                    hi[d] = std::max(hi[d], v[d]);
                }
            }
            key.clear();
            for (int32_t k = a0; k < a1; ++k) {
                const double v[3] = {x[k], y[k], z[k]};
                uint64_t code = 0;
                uint32_t q[3];
                for (int d = 0; d < 3; ++d) {
                    const double span = hi[d] - lo[d];
                    const double t = span > 0 ? (v[d] - lo[d]) / span : 0.0;
                    q[d] = (uint32_t)std::min(1023.0, std::floor(t * 1024.0));
                }
                for (int bit = 9; bit >= 0; --bit)      // Morton (Z-order) interleave
                    for (int d = 0; d < 3; ++d) code = (code << 1) | ((q[d] >> bit) & 1u);
                key.emplace_back(code, k);
            }
            std::stable_sort(key.begin(), key.end(),
                             [](const std::pair<uint64_t, int32_t>& a, const std::pair<uint64_t, int32_t>& c) {
                                 return a.first < c.first;
                             });
            for (int32_t k = a0; k < a1; ++k) order[k] = key[k - a0].second;
        }
        return GBMC_OK;
    } catch (const std::bad_alloc&) {
        return fail(GBMC_ERR_INVALID, "host allocation failed");
    }
}

// Recursive bisection of one system's atoms (indices idx[lo, hi)) along the
// longest side of their bounding box, each cut after a multiple of 64 atoms,
// so that every 64-atom block of the result is one compact leaf.
static void bisect_blocks(const double* x, const double* y, const double* z, int32_t* idx,
                          int32_t lo, int32_t hi)
{
    const int32_t n = hi - lo;
    if (n <= kTile) return;
    double mn[3] = {x[idx[lo]], y[idx[lo]], z[idx[lo]]}, mx[3] = {mn[0], mn[1], mn[2]};
    for (int32_t k = lo; k < hi; ++k) {
        const double v[3] = {x[idx[k]], y[idx[k]], z[idx[k]]};
        for (int d = 0; d < 3; ++d) {
            mn[d] = std::min(mn[d], v[d]);
            mx[d] = std::max(mx[d], v[d]);
        }
    }
    int axis = 0;
    for (int d = 1; d < 3; ++d)
        if (mx[d] - mn[d] > mx[axis] - mn[axis]) axis = d;
    const double* c = axis == 0 ? x : (axis == 1 ? y : z);
    const int32_t nb = (n + kTile - 1) / kTile;
    const int32_t mid = lo + kTile * (nb / 2);
    // ties broken by index, so the order does not depend on the library's nth_element
    std::nth_element(idx + lo, idx + mid, idx + hi, [c](int32_t a, int32_t b) {
        return c[a] < c[b] || (c[a] == c[b] && a < b);
    });
    bisect_blocks(x, y, z, idx, lo, mid);
    bisect_blocks(x, y, z, idx, mid, hi);
}

gbmc_status gbmc_block_order(int32_t n_systems, const int32_t* off, const double* x,
                             const double* y, const double* z, int32_t* order)
{
    try {
        gbmc_status st = check_offsets(n_systems, off);
        if (st != GBMC_OK) return st;
        const int32_t N = n_systems > 0 ? off[n_systems] : 0;
        if (N > 0 && (!x || !y || !z || !order)) return fail(GBMC_ERR_INVALID, "NULL argument");
        for (int32_t k = 0; k < N; ++k)
            if (!std::isfinite(x[k]) || !std::isfinite(y[k]) || !std::isfinite(z[k]))
                return fail(GBMC_ERR_INVALID, "non-finite coordinate");
        for (int32_t k = 0; k < N; ++k) order[k] = k;
        for (int32_t b = 0; b < n_systems; ++b) bisect_blocks(x, y, z, order, off[b], off[b + 1]);
        return GBMC_OK;
    } catch (const std::bad_alloc&) {
        return fail(GBMC_ERR_INVALID, "host allocation failed");
    }
}

// The event pairs for the kernels a call launches (ids), or NULL when the
// timing hook is off.
static hipEvent_t* events(gbmc_plan* p, std::initializer_list<int> ids)
{
    if (!p->timing) return nullptr;
    for (int k : ids) {
        hipEvent_t* e = pool_pair(p, k, p->n_rec[k]++);
        p->cur[2 * k] = e[0];
        p->cur[2 * k + 1] = e[1];
    }
    return p->cur;
}

}  // extern "C"

static bool uses_cutoffs(const GBConst& c) { return c.rgbmax > 0.0 || c.cutoff > 0.0; }

static QueueShape queue_shape(const gbmc_plan* p)
{
    QueueShape sh{};
    for (int k = 0; k < GBMC_N_PASSES; ++k) {
        sh.items[k] = p->d_items[k];
        sh.n_items[k] = p->n_items[k];
    }
    sh.total = p->d_total;
    sh.blocks = p->d_blocks;
    sh.n_blocks = p->n_blocks;
    sh.one_tile = p->tuning.j_blocks_per_item[GBMC_PASS_ENERGY] == 1 &&
                  p->tuning.j_blocks_per_item[GBMC_PASS_CHAIN] == 1;
    sh.spin_limit = p->spin_limit;
    sh.n_cu = p->n_cu;
    return sh;
}

// The three all-pairs passes of a full evaluation as one queued launch
// (staging and output kernels around it); timed as kernel `id` by the timing
// hook.
template <typename T>
static hipError_t run_queued(gbmc_plan* p, const gbmc_atoms* a, const GBConst& c, void* ws,
                             void* born_R, double* e_coul, double* e_gb, void* force, void* dEdq,
                             void* dEdrho, hipStream_t s, int id)
{
    int n = 0;
    for (int k = 0; k < GBMC_N_PASSES; ++k) n += p->n_items[k];
    hipEvent_t* ev = n > 0 ? events(p, {id}) : nullptr;
    return launch_queued<T>(queue_shape(p), p->n_atoms, p->n_sys, (const T*)a->x, (const T*)a->y,
                            (const T*)a->z, (const T*)a->q, (const T*)a->rho,
                            (const T*)a->screen, c, carve<T>(p, ws), (T*)born_R, e_coul, e_gb,
                            (T*)force, (T*)dEdq, (T*)dEdrho, s, ev, id);
}

extern "C" {

// The descreening pass and OBC finalize; with q (the full evaluation) the
// staging also packs the charges and clears the energy and chain passes'
// accumulators, so that the energy call that follows stages nothing.
static hipError_t radii_launch(gbmc_plan* p, const gbmc_atoms* a, const GBConst& c, void* ws,
                               void* born_R, hipStream_t s, bool with_q)
{
    hipEvent_t* ev = p->n_items[GBMC_PASS_RADII] > 0 ? events(p, {kKRadii}) : nullptr;
    if (p->prec == GBMC_FP32_FIXED)
        return launch_radii<float>(p->d_items[GBMC_PASS_RADII], p->n_items[GBMC_PASS_RADII],
                                   p->tuning.waves_per_group[GBMC_PASS_RADII], p->n_atoms,
                                   cut_plan(p), (const float*)a->x, (const float*)a->y,
                                   (const float*)a->z, (const float*)a->rho,
                                   (const float*)a->screen, c, carve<float>(p, ws),
                                   (float*)born_R, s, ev,
                                   with_q ? (const float*)a->q : nullptr);
    return launch_radii<double>(p->d_items[GBMC_PASS_RADII], p->n_items[GBMC_PASS_RADII],
                                p->tuning.waves_per_group[GBMC_PASS_RADII], p->n_atoms,
                                cut_plan(p), (const double*)a->x, (const double*)a->y,
                                (const double*)a->z, (const double*)a->rho,
                                (const double*)a->screen, c, carve<double>(p, ws),
                                (double*)born_R, s, ev, with_q ? (const double*)a->q : nullptr);
}

// The energy pass (and the chain pass when force or dEdrho is requested);
// staged: the preceding radii launch of the same call staged the charges.
static hipError_t energy_launch(gbmc_plan* p, const gbmc_atoms* a, const GBConst& c, void* ws,
                                double* e_coul, double* e_gb, void* force, void* dEdq,
                                void* dEdrho, hipStream_t s, bool staged)
{
    const bool chain = force || dEdrho;
    hipEvent_t* ev = nullptr;
    if (p->n_items[GBMC_PASS_ENERGY] > 0)
        ev = chain ? events(p, {kKEnergy, kKChain}) : events(p, {kKEnergy});
    const PassShape pe{p->d_items[GBMC_PASS_ENERGY], p->n_items[GBMC_PASS_ENERGY],
                       p->tuning.waves_per_group[GBMC_PASS_ENERGY],
                       p->tuning.j_blocks_per_item[GBMC_PASS_ENERGY] == 1};
    const PassShape pc{p->d_items[GBMC_PASS_CHAIN], p->n_items[GBMC_PASS_CHAIN],
                       p->tuning.waves_per_group[GBMC_PASS_CHAIN],
                       p->tuning.j_blocks_per_item[GBMC_PASS_CHAIN] == 1};
    if (p->prec == GBMC_FP32_FIXED)
        return launch_energy_forces<float>(pe, pc, p->n_atoms, p->n_sys, cut_plan(p),
                                           (const float*)a->x, (const float*)a->y,
                                           (const float*)a->z, (const float*)a->q,
                                           (const float*)a->rho, (const float*)a->screen, c,
                                           carve<float>(p, ws), e_coul, e_gb, (float*)force,
                                           (float*)dEdq, (float*)dEdrho, s, ev, staged);
    return launch_energy_forces<double>(pe, pc, p->n_atoms, p->n_sys, cut_plan(p),
                                        (const double*)a->x, (const double*)a->y,
                                        (const double*)a->z, (const double*)a->q,
                                        (const double*)a->rho, (const double*)a->screen, c,
                                        carve<double>(p, ws), e_coul, e_gb, (double*)force,
                                        (double*)dEdq, (double*)dEdrho, s, ev, staged);
}

gbmc_status gb_radii(gbmc_plan* p, const gbmc_atoms* a, const gbmc_gb_params* gp, void* ws,
                     void* born_R, hipStream_t s)
{
    gbmc_status st = check_call(p, a, gp, ws, false);
    if (st != GBMC_OK || p->n_atoms == 0) return st;
    hipError_t e = radii_launch(p, a, make_const(gp), ws, born_R, s, false);
    return e == hipSuccess ? GBMC_OK : hip_fail(e, "gb_radii launch");
}

gbmc_status gb_energy_forces(gbmc_plan* p, const gbmc_atoms* a, const gbmc_gb_params* gp, void* ws,
                             double* e_coul, double* e_gb, void* force, void* dEdq, void* dEdrho,
                             hipStream_t s)
{
    gbmc_status st = check_call(p, a, gp, ws, true);
    if (st != GBMC_OK) return st;
    hipError_t e = energy_launch(p, a, make_const(gp), ws, e_coul, e_gb, force, dEdq, dEdrho, s,
                                 false);
    return e == hipSuccess ? GBMC_OK : hip_fail(e, "gb_energy_forces launch");
}

// A full evaluation: one staging of the inputs for all passes (radii, then
// energies and gradients), or the queued launch in single-launch mode.  With
// fork, that stream is made to wait on the plan's event, recorded on s once
// the Born radii (and the per-atom state of the Monte Carlo calls) are final.
static gbmc_status evaluate_impl(gbmc_plan* p, const gbmc_atoms* a, const gbmc_gb_params* gp,
                                 void* ws, void* born_R, double* e_coul, double* e_gb,
                                 void* force, void* dEdq, void* dEdrho, hipStream_t s,
                                 bool use_fork, hipStream_t fork)
{
    gbmc_status st = check_call(p, a, gp, ws, true);
    if (st != GBMC_OK) return st;
    auto mark = [&]() -> gbmc_status {
        if (!use_fork) return GBMC_OK;
        hipError_t e = hipEventRecord(p->fork_ev, s);
        if (e == hipSuccess) e = hipStreamWaitEvent(fork, p->fork_ev, 0);
        return e == hipSuccess ? GBMC_OK : hip_fail(e, "gb_evaluate_fork: fork event");
    };
    if (p->n_atoms == 0) return mark();
    GBConst c = make_const(gp);
    // in single-launch mode the three all-pairs passes of a full evaluation
    // (forces or dE/drho requested, no cutoffs) run as one queued launch
    const bool chain = force || dEdrho;
    if (p->single_launch && !uses_cutoffs(c) && chain) {
        hipError_t e = p->prec == GBMC_FP32_FIXED
                           ? run_queued<float>(p, a, c, ws, born_R, e_coul, e_gb, force, dEdq,
                                               dEdrho, s, kKEval)
                           : run_queued<double>(p, a, c, ws, born_R, e_coul, e_gb, force, dEdq,
                                                dEdrho, s, kKEval);
        if (e != hipSuccess) return hip_fail(e, "gb_evaluate launch");
        return mark();
    }
    hipError_t e = radii_launch(p, a, c, ws, born_R, s, true);
    if (e != hipSuccess) return hip_fail(e, "gb_evaluate launch");
    st = mark();
    if (st != GBMC_OK) return st;
    e = energy_launch(p, a, c, ws, e_coul, e_gb, force, dEdq, dEdrho, s, true);
    return e == hipSuccess ? GBMC_OK : hip_fail(e, "gb_evaluate launch");
}

gbmc_status gb_evaluate(gbmc_plan* p, const gbmc_atoms* a, const gbmc_gb_params* gp, void* ws,
                        void* born_R, double* e_coul, double* e_gb, void* force, void* dEdq,
                        void* dEdrho, hipStream_t s)
{
    return evaluate_impl(p, a, gp, ws, born_R, e_coul, e_gb, force, dEdq, dEdrho, s, false,
                         nullptr);
}

gbmc_status gb_evaluate_fork(gbmc_plan* p, const gbmc_atoms* a, const gbmc_gb_params* gp,
                             void* ws, void* born_R, double* e_coul, double* e_gb, void* force,
                             void* dEdq, void* dEdrho, hipStream_t s, hipStream_t fork)
{
    if (p && fork == s) return fail(GBMC_ERR_INVALID, "gb_evaluate_fork: fork is the call's stream");
    return evaluate_impl(p, a, gp, ws, born_R, e_coul, e_gb, force, dEdq, dEdrho, s, true, fork);
}

gbmc_status gbmc_plan_set_single_launch(gbmc_plan* p, int32_t enable, int32_t wait_polls)
{
    if (!p) return fail(GBMC_ERR_INVALID, "plan is NULL");
    if (wait_polls < 0) return fail(GBMC_ERR_INVALID, "wait_polls must be >= 0");
    p->single_launch = enable != 0;
    if (wait_polls > 0 || enable) p->spin_limit = wait_polls;
    return GBMC_OK;
}

gbmc_status gb_evaluate_static(gbmc_plan* p, const gbmc_atoms* a, const gbmc_gb_params* gp,
                               void* born_R, double* e_coul, double* e_gb, void* force,
                               void* dEdq, void* dEdrho, hipStream_t s)
{
    if (!p) return fail(GBMC_ERR_INVALID, "plan is NULL");
    if (p->ws_bytes > kScratchBytes)
        return fail(GBMC_ERR_UNSUPPORTED,
                    "gb_evaluate_static: the plan needs " + std::to_string(p->ws_bytes) +
                        " bytes of workspace, more than the library's static scratch of " +
                        std::to_string(kScratchBytes) + " bytes; use gb_evaluate");
    if (!p->scratch) return hip_fail(p->scratch_err, "gb_evaluate_static: static scratch");
    return gb_evaluate(p, a, gp, p->scratch, born_R, e_coul, e_gb, force, dEdq, dEdrho, s);
}

// ------------------------------------------------------------------ sites

gbmc_status gbmc_sites_validate(int32_t n_systems, const int32_t* off, int32_t n_sites,
                                const int32_t* site_system, const int32_t* site_kind,
                                const int32_t* site_atom_offset, const int32_t* site_atoms,
                                const int32_t* site_state_offset,
                                const int32_t* state_charge_offset, const int32_t* state_count)
{
    try {
        gbmc_status st = check_offsets(n_systems, off);
        if (st != GBMC_OK) return st;
        if (n_sites < 0) return fail(GBMC_ERR_INVALID, "n_sites < 0");
        if (n_sites == 0) return GBMC_OK;
        if (!site_system || !site_kind || !site_atom_offset || !site_atoms || !site_state_offset ||
            !state_charge_offset || !state_count)
            return fail(GBMC_ERR_INVALID, "a site table is NULL");
        const int32_t N = n_systems > 0 ? off[n_systems] : 0;
        std::vector<char> used(N, 0);
        if (site_atom_offset[0] != 0 || site_state_offset[0] != 0 || state_charge_offset[0] != 0)
            return fail(GBMC_ERR_INVALID, "site CSR offsets must start at 0");
        for (int32_t m = 0; m < n_sites; ++m) {
            const int32_t b = site_system[m];
            if (b < 0 || b >= n_systems) return fail(GBMC_ERR_INVALID, "site_system out of range");
            if (m > 0 && b < site_system[m - 1]) return fail(GBMC_ERR_INVALID, "site_system must be non-decreasing");
            if (site_kind[m] != 0 && site_kind[m] != 1) return fail(GBMC_ERR_INVALID, "site_kind must be 0 or 1");
            const int32_t na = site_atom_offset[m + 1] - site_atom_offset[m];
            if (na < 1) return fail(GBMC_ERR_INVALID, "a site needs at least one atom");
            if (na > kMaxSiteAtoms) return fail(GBMC_ERR_UNSUPPORTED, "a site has more than 256 atoms");
            for (int32_t k = site_atom_offset[m]; k < site_atom_offset[m + 1]; ++k) {
                const int32_t g = site_atoms[k];
                if (g < off[b] || g >= off[b + 1]) return fail(GBMC_ERR_INVALID, "site atom outside its system");
                if (used[g]) return fail(GBMC_ERR_INVALID, "sites overlap (an atom belongs to two sites)");
                used[g] = 1;
            }
            const int32_t ns = site_state_offset[m + 1] - site_state_offset[m];
            if (ns < 2 || ns > kMaxStates) return fail(GBMC_ERR_UNSUPPORTED, "a site needs 2..8 states");
            for (int32_t g = site_state_offset[m]; g < site_state_offset[m + 1]; ++g) {
                if (state_charge_offset[g + 1] - state_charge_offset[g] != na)
                    return fail(GBMC_ERR_INVALID, "a state charge row does not match its site's atom count");
                if (state_count[g] < 0) return fail(GBMC_ERR_INVALID, "state_count must be >= 0");
            }
        }
        return GBMC_OK;
    } catch (const std::bad_alloc&) {
        return fail(GBMC_ERR_INVALID, "host allocation failed");
    }
}

gbmc_status gbmc_sites_create(gbmc_plan* p, gbmc_sites** out, int32_t n_sites,
                              const int32_t* site_system, const int32_t* site_kind,
                              const int32_t* site_atom_offset, const int32_t* site_atoms,
                              const int32_t* site_state_offset, const int32_t* state_charge_offset,
                              const double* state_charges, const double* state_gref,
                              const int32_t* state_count)
{
    try {
        if (!out) return fail(GBMC_ERR_INVALID, "sites out-pointer is NULL");
        *out = nullptr;
        if (!p) return fail(GBMC_ERR_INVALID, "plan is NULL");
        gbmc_status st = gbmc_sites_validate(p->n_sys, p->offset.data(), n_sites, site_system, site_kind,
                                             site_atom_offset, site_atoms, site_state_offset,
                                             state_charge_offset, state_count);
        if (st != GBMC_OK) return st;
        if (n_sites > 0 && (!state_charges || !state_gref))
            return fail(GBMC_ERR_INVALID, "state_charges or state_gref is NULL");
        const int32_t B = p->n_sys;
        const int32_t S = n_sites;
        const int32_t n_sa = S > 0 ? site_atom_offset[S] : 0;
        const int32_t n_st = S > 0 ? site_state_offset[S] : 0;
        const int32_t n_q = n_st > 0 ? state_charge_offset[n_st] : 0;
        std::vector<int32_t> cand(S + 1, 0), prot_off(B + 1, 0), redox_off(B + 1, 0), prot, redox;
        std::vector<int32_t> sys_sa(B + 1, 0);
        for (int32_t m = 0; m < S; ++m)
            cand[m + 1] = cand[m] + (site_state_offset[m + 1] - site_state_offset[m] - 1);
        // per-system site lists and site-atom ranges
        std::vector<int32_t> first(B, -1), last(B, -1);
        for (int32_t m = 0; m < S; ++m) {
            int32_t b = site_system[m];
            if (first[b] < 0) first[b] = m;
            last[b] = m;
        }
        for (int32_t b = 0; b < B; ++b) {
            for (int32_t m = 0; m < S; ++m)
                if (site_system[m] == b) (site_kind[m] == 0 ? prot : redox).push_back(m);
            prot_off[b + 1] = (int32_t)prot.size();
            redox_off[b + 1] = (int32_t)redox.size();
            sys_sa[b] = first[b] >= 0 ? site_atom_offset[first[b]] : (b > 0 ? sys_sa[b - 1] : 0);
        }
        // sys_sa must be monotone: recompute as a running boundary
        for (int32_t b = 0; b < B; ++b) sys_sa[b + 1] = last[b] >= 0 ? site_atom_offset[last[b] + 1] : sys_sa[b];
        for (int32_t b = 0; b < B; ++b)
            if (first[b] < 0) sys_sa[b] = sys_sa[b + 1];
        // FP64 potential-row items: (64 site atoms) x (kPhiChunk atoms) per system;
        // each adds into the flattened site-atom slots of its 64 site atoms
        std::vector<RowItem> rows;
        for (int32_t b = 0; b < B; ++b) {
            const int32_t na = sys_sa[b + 1] - sys_sa[b];
            if (na == 0) continue;
            const int32_t n = p->offset[b + 1] - p->offset[b];
            const int32_t chunks = (n + kPhiChunk - 1) / kPhiChunk;
            for (int32_t c = 0; c < chunks; ++c)
                for (int32_t s0 = 0; s0 < na; s0 += kTile) {
                    RowItem r{};
                    r.base = p->offset[b];
                    r.n = n;
                    r.sa0 = sys_sa[b] + s0;
                    r.sa1 = sys_sa[b] + std::min(na, s0 + kTile);
                    r.j0 = c * kPhiChunk;
                    r.j1 = std::min(n, (c + 1) * kPhiChunk);
                    r.out = sys_sa[b] + s0;
                    rows.push_back(r);
                }
        }
        // one device allocation for every table
        size_t o = 0;
        auto seg = [&](size_t bytes) { size_t at = o; o = align256(o + bytes); return at; };
        size_t o_sys = seg(4 * S), o_kind = seg(4 * S), o_sao = seg(4 * (S + 1)), o_sa = seg(4 * n_sa),
               o_sso = seg(4 * (S + 1)), o_sco = seg(4 * (n_st + 1)), o_q = seg(8 * n_q),
               o_gref = seg(8 * n_st), o_cnt = seg(4 * n_st), o_cand = seg(4 * (S + 1)),
               o_po = seg(4 * (B + 1)), o_ps = seg(4 * prot.size()), o_ro = seg(4 * (B + 1)),
               o_rs = seg(4 * redox.size()), o_syssa = seg(4 * (B + 1)),
               o_rows = seg(sizeof(RowItem) * rows.size());
        std::vector<char> h(o, 0);
        auto put = [&](size_t at, const void* src, size_t bytes) { if (bytes) std::memcpy(h.data() + at, src, bytes); };
        if (S > 0) {
            put(o_sys, site_system, 4 * S);
            put(o_kind, site_kind, 4 * S);
            put(o_sao, site_atom_offset, 4 * (S + 1));
            put(o_sa, site_atoms, 4 * n_sa);
            put(o_sso, site_state_offset, 4 * (S + 1));
            put(o_sco, state_charge_offset, 4 * (n_st + 1));
            put(o_q, state_charges, 8 * n_q);
            put(o_gref, state_gref, 8 * n_st);
            put(o_cnt, state_count, 4 * n_st);
        }
        put(o_cand, cand.data(), 4 * (S + 1));
        put(o_po, prot_off.data(), 4 * (B + 1));
        put(o_ps, prot.data(), 4 * prot.size());
        put(o_ro, redox_off.data(), 4 * (B + 1));
        put(o_rs, redox.data(), 4 * redox.size());
        put(o_syssa, sys_sa.data(), 4 * (B + 1));
        put(o_rows, rows.data(), sizeof(RowItem) * rows.size());
        auto* sp = new gbmc_sites();
        sp->plan = p;
        sp->n_sites = S;
        sp->n_cand = cand[S];
        sp->n_rowitems = (int32_t)rows.size();
        sp->n_site_atoms = (size_t)n_sa;
        for (int32_t b = 0; b < B; ++b) {
            sp->max_sys_site_atoms = std::max(sp->max_sys_site_atoms, sys_sa[b + 1] - sys_sa[b]);
            sp->max_sys_sites = std::max({sp->max_sys_sites, prot_off[b + 1] - prot_off[b],
                                          redox_off[b + 1] - redox_off[b]});
        }
        hipError_t e = hipMalloc(&sp->d_mem, std::max<size_t>(o, 256));
        if (e != hipSuccess) { delete sp; return hip_fail(e, "hipMalloc(site tables)"); }
        e = hipMemcpy(sp->d_mem, h.data(), o, hipMemcpyHostToDevice);
        if (e != hipSuccess) { (void)hipFree(sp->d_mem); delete sp; return hip_fail(e, "hipMemcpy(site tables)"); }
        char* d = static_cast<char*>(sp->d_mem);
        SiteDev& sd = sp->dev;
        sd.n_sites = S;
        sd.n_cand = cand[S];
        sd.n_rowitems = (int32_t)rows.size();
        sd.n_site_atoms = (int32_t)n_sa;
        sd.site_system = (const int32_t*)(d + o_sys);
        sd.site_kind = (const int32_t*)(d + o_kind);
        sd.site_atom_offset = (const int32_t*)(d + o_sao);
        sd.site_atoms = (const int32_t*)(d + o_sa);
        sd.site_state_offset = (const int32_t*)(d + o_sso);
        sd.state_charge_offset = (const int32_t*)(d + o_sco);
        sd.state_charges = (const double*)(d + o_q);
        sd.state_gref = (const double*)(d + o_gref);
        sd.state_count = (const int32_t*)(d + o_cnt);
        sd.cand_offset = (const int32_t*)(d + o_cand);
        sd.sys_prot_offset = (const int32_t*)(d + o_po);
        sd.sys_prot_sites = (const int32_t*)(d + o_ps);
        sd.sys_redox_offset = (const int32_t*)(d + o_ro);
        sd.sys_redox_sites = (const int32_t*)(d + o_rs);
        sd.site_sa_offset = sd.site_atom_offset;
        sd.sys_sa_offset = (const int32_t*)(d + o_syssa);
        sd.rowitems = (const RowItem*)(d + o_rows);
        *out = sp;
        return GBMC_OK;
    } catch (const std::bad_alloc&) {
        return fail(GBMC_ERR_INVALID, "host allocation failed");
    }
}

void gbmc_sites_destroy(gbmc_sites* s)
{
    if (!s) return;
    if (s->d_mem) (void)hipFree(s->d_mem);
    delete s;
}

int32_t gbmc_sites_n_candidates(const gbmc_sites* s) { return s ? s->n_cand : 0; }

size_t gbmc_sites_workspace_bytes(const gbmc_sites* s)
{
    return s ? align256(std::max<size_t>(8 * s->n_site_atoms, 8)) : 0;
}

static gbmc_status check_sites(const gbmc_plan* p, const gbmc_sites* s, const void* sws)
{
    if (!s) return fail(GBMC_ERR_INVALID, "sites is NULL");
    if (s->plan != p) return fail(GBMC_ERR_INVALID, "sites were created for another plan");
    if (s->n_site_atoms > 0 && !sws) return fail(GBMC_ERR_INVALID, "site workspace is NULL");
    return GBMC_OK;
}

gbmc_status mc_state_dE(gbmc_plan* p, const gbmc_sites* s, const gbmc_atoms* a,
                        const gbmc_gb_params* gp, void* ws, void* sws, const int32_t* current_state,
                        const double* pH, const double* E_volt, double T, double* dE, double* dG,
                        hipStream_t stream)
{
    gbmc_status st = check_call(p, a, gp, ws, true);
    if (st != GBMC_OK) return st;
    st = check_sites(p, s, sws);
    if (st != GBMC_OK) return st;
    if (s->n_sites == 0) return GBMC_OK;
    if (!current_state || !dE || !pH || !E_volt) return fail(GBMC_ERR_INVALID, "a Monte Carlo array is NULL");
    if (!(T > 0.0) || !std::isfinite(T)) return fail(GBMC_ERR_INVALID, "temperature must be > 0");
    GBConst c = make_const(gp);
    hipEvent_t* ev = s->dev.n_rowitems > 0 ? events(p, {kKSiteRows, kKSiteDE}) : events(p, {kKSiteDE});
    hipError_t e;
    if (p->prec == GBMC_FP32_FIXED)
        e = launch_state_dE<float>(s->dev, p->n_atoms, (const float*)a->x, (const float*)a->y, (const float*)a->z,
                                   (const float*)a->q, c, carve<float>(p, ws), (unsigned long long*)sws,
                                   current_state, pH, E_volt, T, dE, dG, stream, ev);
    else
        e = launch_state_dE<double>(s->dev, p->n_atoms, (const double*)a->x, (const double*)a->y,
                                    (const double*)a->z, (const double*)a->q, c, carve<double>(p, ws),
                                    (unsigned long long*)sws, current_state, pH, E_volt, T, dE, dG, stream, ev);
    return e == hipSuccess ? GBMC_OK : hip_fail(e, "mc_state_dE launch");
}

gbmc_status mc_step(gbmc_plan* p, const gbmc_sites* s, const gbmc_atoms* a, void* q,
                    const gbmc_gb_params* gp, void* ws, void* sws, int32_t* current_state,
                    const double* pH, const double* E_volt, double T, const double* dE,
                    const double* dG, const double* u, int32_t* n_electrons, int64_t* counters,
                    int32_t* accepted, hipStream_t stream)
{
    gbmc_status st = check_call(p, a, gp, ws, false);
    if (st != GBMC_OK) return st;
    st = check_sites(p, s, sws);
    if (st != GBMC_OK) return st;
    if (p->n_sys == 0) return GBMC_OK;
    if (s->n_sites > 0 && (!q || !current_state || !dE || !dG || !u || !pH || !E_volt))
        return fail(GBMC_ERR_INVALID, "a Monte Carlo array is NULL");
    if (!u) return fail(GBMC_ERR_INVALID, "uniforms are NULL");
    if (!(T > 0.0) || !std::isfinite(T)) return fail(GBMC_ERR_INVALID, "temperature must be > 0");
    GBConst c = make_const(gp);
    hipEvent_t* ev = events(p, {kKMCStep});
    hipError_t e;
    if (p->prec == GBMC_FP32_FIXED)
        e = launch_mc_step<float>(s->dev, p->n_sys, (const float*)a->x, (const float*)a->y,
                                  (const float*)a->z, (float*)q, c, carve<float>(p, ws), current_state,
                                  pH, E_volt, T, dE, dG, u, n_electrons, counters, accepted, stream, ev);
    else
        e = launch_mc_step<double>(s->dev, p->n_sys, (const double*)a->x, (const double*)a->y,
                                   (const double*)a->z, (double*)q, c, carve<double>(p, ws),
                                   current_state, pH, E_volt, T, dE, dG, u, n_electrons, counters,
                                   accepted, stream, ev);
    return e == hipSuccess ? GBMC_OK : hip_fail(e, "mc_step launch");
}

gbmc_status mc_sweep(gbmc_plan* p, const gbmc_sites* s, const gbmc_atoms* a, void* q,
                     const gbmc_gb_params* gp, void* ws, void* sws, int32_t* current_state,
                     const double* pH, const double* E_volt, double T, int32_t kinds,
                     const double* u, int32_t* n_electrons, int64_t* counters, int32_t* accepted,
                     double* dG, hipStream_t stream)
{
    gbmc_status st = check_call(p, a, gp, ws, true);
    if (st != GBMC_OK) return st;
    st = check_sites(p, s, sws);
    if (st != GBMC_OK) return st;
    if (kinds < 0 || kinds > 3) return fail(GBMC_ERR_INVALID, "kinds must be 0..3 (bit 0 protonation, bit 1 redox)");
    if (p->n_sys == 0 || s->n_sites == 0) return GBMC_OK;
    if (!q || !current_state || !u || !pH || !E_volt)
        return fail(GBMC_ERR_INVALID, "a Monte Carlo array is NULL");
    if (!(T > 0.0) || !std::isfinite(T)) return fail(GBMC_ERR_INVALID, "temperature must be > 0");
    if (s->max_sys_site_atoms > kMaxSweepSiteAtoms || s->max_sys_sites > kMaxSweepSites)
        return fail(GBMC_ERR_UNSUPPORTED, "mc_sweep supports at most 1024 site atoms and 1024 "
                                          "sites of one kind per system");
    GBConst c = make_const(gp);
    hipError_t e;
    if (p->prec == GBMC_FP32_FIXED)
        e = launch_mc_sweep<float>(s->dev, p->n_sys, s->max_sys_site_atoms, (const float*)a->x,
                                   (const float*)a->y, (const float*)a->z, (const float*)a->q,
                                   (float*)q, c, carve<float>(p, ws), (unsigned long long*)sws,
                                   current_state, pH, E_volt, T, kinds, u, n_electrons, counters,
                                   accepted, dG, stream);
    else
        e = launch_mc_sweep<double>(s->dev, p->n_sys, s->max_sys_site_atoms, (const double*)a->x,
                                    (const double*)a->y, (const double*)a->z, (const double*)a->q,
                                    (double*)q, c, carve<double>(p, ws), (unsigned long long*)sws,
                                    current_state, pH, E_volt, T, kinds, u, n_electrons, counters,
                                    accepted, dG, stream);
    return e == hipSuccess ? GBMC_OK : hip_fail(e, "mc_sweep launch");
}

gbmc_status remd_exchange(int32_t M, const double* E_rung, const int32_t* Ne, int32_t* rep, double T,
                          int32_t parity, int32_t wrap, const double* u, int32_t* accepted,
                          double* E_of_rep, hipStream_t stream)
{
    if (M < 0) return fail(GBMC_ERR_INVALID, "n_rep < 0");
    if (parity != 0 && parity != 1) return fail(GBMC_ERR_INVALID, "parity must be 0 or 1");
    if (!(T > 0.0) || !std::isfinite(T)) return fail(GBMC_ERR_INVALID, "temperature must be > 0");
    if (M < 2) return GBMC_OK;
    if (!E_rung || !Ne || !rep || !u) return fail(GBMC_ERR_INVALID, "an exchange array is NULL");
    hipError_t e = launch_remd_exchange(M, E_rung, Ne, rep, T, parity, wrap, u, accepted, E_of_rep, stream);
    return e == hipSuccess ? GBMC_OK : hip_fail(e, "remd_exchange launch");
}

gbmc_status md_langevin_step(gbmc_plan* p, void* x, void* y, void* z, void* v, const void* force,
                             const void* inv_mass, const void* xi, const void* xref, double k_restr,
                             double dt, double gamma, double T, hipStream_t stream)
{
    if (!p) return fail(GBMC_ERR_INVALID, "plan is NULL");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(GBMC_ERR_INVALID, "dt must be > 0");
    if (!(gamma >= 0.0) || !std::isfinite(gamma)) return fail(GBMC_ERR_INVALID, "gamma must be >= 0");
    if (!(T >= 0.0) || !std::isfinite(T)) return fail(GBMC_ERR_INVALID, "temperature must be >= 0");
    if (!(k_restr >= 0.0) || !std::isfinite(k_restr))
        return fail(GBMC_ERR_INVALID, "restraint constant must be >= 0");
    if (p->n_atoms == 0) return GBMC_OK;
    if (!x || !y || !z || !v || !force || !inv_mass || !xi)
        return fail(GBMC_ERR_INVALID, "a dynamics array is NULL");
    hipError_t e;
    if (p->prec == GBMC_FP32_FIXED)
        e = launch_md_langevin<float>(p->n_atoms, (float*)x, (float*)y, (float*)z, (float*)v,
                                      (const float*)force, (const float*)inv_mass, (const float*)xi,
                                      (const float*)xref, k_restr, dt, gamma, T, stream);
    else
        e = launch_md_langevin<double>(p->n_atoms, (double*)x, (double*)y, (double*)z, (double*)v,
                                       (const double*)force, (const double*)inv_mass,
                                       (const double*)xi, (const double*)xref, k_restr, dt, gamma,
                                       T, stream);
    return e == hipSuccess ? GBMC_OK : hip_fail(e, "md_langevin_step launch");
}

size_t gb_plain_workspace_bytes(int32_t n_atoms)
{
    return n_atoms > 0 ? plain_workspace_bytes(n_atoms) : 0;
}

gbmc_status gb_plain_fp64(int32_t n_systems, const int32_t* host_atom_offset,
                          const int32_t* atom_offset, const gbmc_atoms* a,
                          const gbmc_gb_params* gp, void* workspace, double* born_R,
                          double* e_coul, double* e_gb, double* force, double* dEdq,
                          double* dEdrho, hipStream_t stream)
{
    gbmc_status st = check_offsets(n_systems, host_atom_offset);
    if (st != GBMC_OK) return st;
    if (!a || !gp) return fail(GBMC_ERR_INVALID, "NULL argument");
    st = gbmc_params_validate(gp);
    if (st != GBMC_OK) return st;
    if (gp->kappa != 0.0 || gp->rgbmax != 0.0 || gp->cutoff != 0.0)
        return fail(GBMC_ERR_UNSUPPORTED, "the plain FP64 form has no salt and no cutoffs");
    const int32_t N = n_systems > 0 ? host_atom_offset[n_systems] : 0;
    if (n_systems > 0 && !atom_offset) return fail(GBMC_ERR_INVALID, "atom_offset is NULL");
    if (N > 0 && (!a->x || !a->y || !a->z || !a->q || !a->rho || !a->screen || !workspace))
        return fail(GBMC_ERR_INVALID, "an input array or the workspace is NULL");
    hipError_t e = launch_plain_fp64(n_systems, atom_offset, N, (const double*)a->x,
                                     (const double*)a->y, (const double*)a->z, (const double*)a->q,
                                     (const double*)a->rho, (const double*)a->screen, make_const(gp),
                                     workspace, born_R, e_coul, e_gb, force, dEdq, dEdrho, stream);
    return e == hipSuccess ? GBMC_OK : hip_fail(e, "gb_plain_fp64 launch");
}

gbmc_status gbmc_check_overflow(const gbmc_plan* p, void* ws, hipStream_t s, int32_t* flag)
{
    if (!p || !flag) return fail(GBMC_ERR_INVALID, "NULL argument");
    if (!ws) ws = p->scratch;     // the static scratch of gb_evaluate_static
    if (!ws) return fail(GBMC_ERR_INVALID, "workspace is NULL");
    // two words: [0] a fixed-point accumulator overflowed, [1] a dependency
    // wait of a queued launch gave up (its results are not valid)
    int* d = reinterpret_cast<int*>(static_cast<char*>(ws) + p->off_ovf);
    int h[2] = {0, 0};
    hipError_t e = hipMemcpyAsync(h, d, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "gbmc_check_overflow");
    *flag = (h[0] || h[1]) ? 1 : 0;
    if (*flag) {
        const int zero[2] = {0, 0};
        e = hipMemcpyAsync(d, zero, sizeof(zero), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "gbmc_check_overflow");
        if (h[1])
            return fail(GBMC_ERR_HIP, "a dependency wait of a queued launch gave up "
                                      "(see gbmc_plan_set_wait_limit); the results are not valid");
        return fail(GBMC_ERR_OVERFLOW, "a fixed-point accumulator overflowed");
    }
    return GBMC_OK;
}

}  // extern "C"
