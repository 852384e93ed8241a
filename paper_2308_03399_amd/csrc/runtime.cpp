// Host runtime and C ABI of the multi-shot noisy state-vector library.
//
// sv_run_circuit: validate -> expand noise sites (rules attached after each
// matching gate, in rule order; Sec. III-B) -> device op records with FP64
// matrices -> static pass plan (groups of consecutive ops whose qubits fit
// in one LDS tile) -> upload -> persistent executor launch (plus waiting-
// list relaunches in branch mode, Sec. IV-B) -> device histogram of the
// classical registers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <list>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/svbatch.h"
#include "program.h"

using namespace svb;
using cd = std::complex<double>;

extern "C" {
hipError_t svb_launch_init(const ExecParams *P, int restart, int n_root, int root_slot,
                           int n_free, hipStream_t st);
hipError_t svb_launch_restart(const ExecParams *P, int n_wait, hipStream_t st);
hipError_t svb_launch_exec(const ExecParams *P, int is_c128, int reg_bits, int workers,
                           hipStream_t st);
hipError_t svb_exec_occupancy(int is_c128, int tile_q, int resident, int reg_bits, int nbuf,
                              int stage_cap, int *blocks_per_cu);
size_t svb_exec_lds_bytes(int tile_q, int amp_bytes, int resident, int nbuf, int stage_cap);
hipError_t svb_counts(const uint64_t *memory, int64_t n, void *temp, size_t temp_bytes,
                      uint64_t *keys_sorted, uint64_t *uniq, uint32_t *cnt, uint32_t *n_uniq,
                      hipStream_t st);
size_t svb_counts_temp_bytes(int64_t n);
hipError_t svb_noalloc_scratch(void **ptr, uint64_t *bytes);
hipError_t svb_graph_nodes(const ExecParams *P, int is_c128, int reg_bits, int workers,
                           void **init_fn, unsigned *init_grid, void **exec_fn,
                           unsigned *exec_grid, unsigned *block, size_t *exec_lds);
hipError_t svb_plain_run(int is_c128, const DevOp *ops, const DevOp *hops, int n_ops,
                         const DevRule *rules, const DevRule *hrules, const double *pool, int n,
                         uint64_t n_shots, uint64_t shot_base, uint64_t seed, void *state,
                         uint64_t *memory, uint64_t *margins, double *partial, int red_blocks,
                         double *chunk, void *cell, double ro01, double ro10, hipStream_t st);
}

// ------------------------------------------------------------------ errors
static thread_local std::string g_err;

static sv_status fail(sv_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

#define HIPCHK(expr)                                                              \
    do {                                                                          \
        hipError_t _e = (expr);                                                   \
        if (_e != hipSuccess)                                                     \
            return fail(SV_EDEVICE, "%s: %s", #expr, hipGetErrorString(_e));      \
    } while (0)

static uint64_t align_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

// HIP events time a run; a handle without events (the no-allocation entry
// point) skips the timing and waits on its stream instead.
static hipError_t ev_record(hipEvent_t e, hipStream_t s) { return e ? hipEventRecord(e, s) : hipSuccess; }
static hipError_t ev_wait(hipEvent_t e, hipStream_t s)
{
    return e ? hipEventSynchronize(e) : hipStreamSynchronize(s);
}
static hipError_t ev_ms(float *ms, hipEvent_t a, hipEvent_t b)
{
    *ms = 0;
    return (a && b) ? hipEventElapsedTime(ms, a, b) : hipSuccess;
}

constexpr int kPlainRedBlocks = 1024;  // blocks of a plain-mode reduction

// ------------------------------------------------------------------ handle
struct Plan {
    std::vector<uint32_t> order;  // device position -> expanded index
    std::vector<PassInfo> passes;
    std::vector<GroupInfo> groups;
    std::vector<uint32_t> op_pass, op_group;  // per device position
};

// Pass plans of recent circuits, keyed by the structural signature each was
// made from (planning depends on nothing else), shared by every handle of
// the process: a job run as waves or serving chunks on fresh handles plans
// once. At most kPlanCacheEntries, least recently used dropped first.
struct PlanEntry {
    std::vector<int32_t> sig;
    Plan plan;
};
constexpr size_t kPlanCacheEntries = 8;
static std::mutex g_plan_mu;
static std::list<PlanEntry> g_plans;  // most recently used first

static bool plan_lookup(const std::vector<int32_t> &sig, Plan &out)
{
    std::lock_guard<std::mutex> lk(g_plan_mu);
    for (auto it = g_plans.begin(); it != g_plans.end(); ++it) {
        if (it->sig != sig) continue;
        out = it->plan;
        g_plans.splice(g_plans.begin(), g_plans, it);
        return true;
    }
    return false;
}

static void plan_store(std::vector<int32_t> &&sig, const Plan &plan)
{
    std::lock_guard<std::mutex> lk(g_plan_mu);
    for (const PlanEntry &e : g_plans)
        if (e.sig == sig) return;
    g_plans.push_front(PlanEntry{std::move(sig), plan});
    if (g_plans.size() > kPlanCacheEntries) g_plans.pop_back();
}

struct sv_batch {
    int n = 0;
    int64_t shots = 0;
    sv_dtype dtype = SV_C64;
    // options
    int mode = SV_MODE_BATCH;
    int64_t opt_slots = 0, opt_workers = 0, opt_tile = 0;
    int64_t program_bytes = 8 << 20;
    int64_t dump_shot = -1;
    int64_t spin_ms = 300000;
    int64_t spin_elapsed = 0;         // 1: the wait bound counts elapsed time, not stalled time
    int64_t shot_offset = 0;
    // derived
    int tile_q = 0, resident = 0, workers = 0, slots = 0;
    int use_groups = 0, reg_bits = 0;  // register-group engine, log2(amps per thread)
    int64_t opt_engine = 0;            // 0 automatic, 1 LDS sweeps only
    int64_t opt_pipeline = -1;         // -1 automatic, 0 one tile buffer, 1 two
    int nbuf = 1;                      // LDS tile buffers of grouped streamed passes
    int stage_cap = 0;                 // ops of a pass staged in LDS (resident register groups)
    int cus = 0;
    int64_t wallclock_khz = 100000;
    int64_t auto_slots = 0;            // branch mode's automatic slot count, fixed at first sizing
    int64_t auto_workers = 0;          // batch mode's memory-bounded worker count, same
    bool no_counts = false;            // no room reserved for the counts histogram
    int64_t opt_graph = 0;             // 1: launches replayed from a HIP graph
    int64_t opt_mfma = 0;              // 0 automatic, 1 vector ALU, 2 matrix cores
    int mfma = 0;                      // the last program's choice
    bool noalloc_run = false;          // inside sv_run_circuit_noalloc
    hipGraph_t graph = nullptr;        // [init kernel] -> [executor]
    hipGraphExec_t gexec = nullptr;
    hipGraphNode_t n_init = nullptr, n_exec = nullptr;
    const void *graph_fn = nullptr;    // executor instantiation, grid and LDS the graph holds
    unsigned graph_grid = 0;
    size_t graph_lds = 0;
    uint64_t prog_hash = 0;            // program last uploaded by a graph run (0: none)
    char *prog_arena = nullptr;        // arena it was uploaded to
    // arena
    bool attached = false;
    char *arena = nullptr;
    uint64_t arena_bytes = 0;
    hipStream_t stream = nullptr;
    struct Layout {
        uint64_t prog, memory, margins, perm, tmp, waiting, queue, ready, ctl, free_slots, tile_sums,
            dump, counts_tmp, keys_sorted, uniq, cnt, nuniq, slots, total;
    } lay{};
    // results
    bool have_results = false;
    bool have_stats = false;
    bool have_dump = false;
    sv_stats stats{};
    hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr, ev3 = nullptr;
};

static int amp_bytes(const sv_batch *b) { return b->dtype == SV_C128 ? 16 : 8; }
static uint64_t state_bytes(const sv_batch *b) { return (uint64_t)amp_bytes(b) << b->n; }

// tile buffers when the caller leaves the choice to the library
constexpr int kAutoTileBuffers = 1;

static sv_status derive(sv_batch *b)
{
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, dev));
    b->cus = prop.multiProcessorCount;
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
        b->wallclock_khz = khz;
    // largest tile whose LDS footprint fits one workgroup on this device
    size_t lds_cap = prop.sharedMemPerBlockOptin > 0 ? prop.sharedMemPerBlockOptin
                                                     : prop.sharedMemPerBlock;
    if (prop.maxSharedMemoryPerMultiProcessor > 0)
        lds_cap = std::min(lds_cap, (size_t)prop.maxSharedMemoryPerMultiProcessor);
    const size_t static_lds = 0;  // the executor keeps all its LDS state in the dynamic block
    // two tile buffers: the next tile is fetched into LDS while the
    // current one computes, one workgroup per compute unit at the largest
    // tile; one buffer: two workgroups per compute unit overlap instead
    int nbuf = b->opt_pipeline == 0 ? 1 : (b->opt_pipeline == 1 ? 2 : kAutoTileBuffers);
    auto fits = [&](int kk, int nb, int per_cu) {
        return (size_t)per_cu * (svb_exec_lds_bytes(kk, amp_bytes(b), 0, nb, 0) + static_lds) <= lds_cap;
    };
    int kmax = b->dtype == SV_C128 ? 13 : kMaxTileQ;
    while (kmax > 6 && !fits(kmax, nbuf, 1)) --kmax;
    int kdef = kmax;
    if (nbuf == 1)
        while (kdef > 6 && !fits(kdef, 1, 2)) --kdef;
    int k = b->opt_tile > 0 ? (int)b->opt_tile : kdef;
    if (k > kmax) {
        if (b->opt_pipeline != 1 && fits(k, 1, 1)) nbuf = 1;  // a larger tile wins over the pipeline
        else k = kmax;
    }
    if (b->n <= k) {
        b->resident = 1;
        b->tile_q = b->n;
    } else {
        b->resident = 0;
        b->tile_q = k;
    }
    // register groups need 2^k = kWG * 2^r amplitudes per tile. A state
    // resident in LDS uses them from 4 amplitudes per thread (10 qubits) on
    // when its passes can be staged in LDS (states of at most 32 KiB) or
    // when asked for (engine 2); larger resident states run their ops as
    // LDS sweeps by default, which measured faster without staging
    const int r = b->tile_q - kWGBits;
    const bool small = state_bytes(b) <= (32u << 10);
    const bool r_ok = b->resident ? (r >= 2 && r <= 5 && (b->opt_engine == 2 || small))
                                  : (b->dtype == SV_C128 ? (r == 4 || r == 5) : (r >= 4 && r <= 6));
    b->use_groups = (r_ok && b->opt_engine != 1) ? 1 : 0;
    b->reg_bits = b->use_groups ? r : 0;
    b->nbuf = (b->use_groups && !b->resident) ? nbuf : 1;
    // a resident state planned into register groups copies each pass's op
    // records to LDS first, when the state is small enough to leave room
    b->stage_cap = (b->use_groups && b->resident && state_bytes(b) <= (32u << 10)) ? kStageOps : 0;
    if (b->mode == SV_MODE_PLAIN) {  // one state, per-op kernels over the whole GPU
        b->use_groups = 0;
        b->reg_bits = 0;
        b->workers = 1;
        b->slots = 1;
        return SV_OK;
    }
    int per_cu = 0;
    HIPCHK(svb_exec_occupancy(b->dtype == SV_C128, b->tile_q, b->resident, b->reg_bits, b->nbuf,
                              b->stage_cap,
                              &per_cu));
    if (per_cu < 1) return fail(SV_EDEVICE, "executor does not fit on a compute unit");
    int64_t w = b->opt_workers > 0 ? b->opt_workers : (int64_t)per_cu * b->cus;
    if (b->mode == SV_MODE_BATCH) w = std::min<int64_t>(w, b->shots);
    // batch mode keeps one state per workgroup: the automatic count also
    // stays within 80% of the free device memory (decided once, so the
    // footprint and the attach agree)
    if (b->mode == SV_MODE_BATCH && !b->resident && b->opt_workers <= 0) {
        if (b->auto_workers == 0) {
            int64_t cap = w;
            size_t free_b = 0, total_b = 0;
            if (hipMemGetInfo(&free_b, &total_b) == hipSuccess)
                cap = (int64_t)((double)free_b * 0.8 / (double)state_bytes(b));
            b->auto_workers = std::max<int64_t>(1, std::min<int64_t>(w, cap));
        }
        w = b->auto_workers;
    }
    b->workers = (int)std::max<int64_t>(1, w);
    // state slots
    if (b->resident) {
        b->slots = b->mode == SV_MODE_BRANCH
                       ? (int)(b->opt_slots > 0 ? b->opt_slots
                                                : std::min<int64_t>(b->shots, 4 * (int64_t)b->workers))
                       : 0;
    } else if (b->mode == SV_MODE_BRANCH) {
        // automatic: one slot per shot while they fit in half the free
        // device memory (no waiting list), at least two per workgroup
        // (decided once, so the footprint and the attach agree)
        if (b->opt_slots <= 0 && b->auto_slots == 0) {
            int64_t want = 2 * (int64_t)b->workers;
            size_t free_b = 0, total_b = 0;
            if (hipMemGetInfo(&free_b, &total_b) == hipSuccess)
                want = std::max<int64_t>(want, (int64_t)(free_b / 2 / state_bytes(b)));
            b->auto_slots = std::min<int64_t>({b->shots, want, (int64_t)1 << 24});
        }
        b->slots = (int)(b->opt_slots > 0 ? b->opt_slots : b->auto_slots);
        b->slots = std::max(b->slots, 1);
    } else {
        b->slots = b->workers;
    }
    return SV_OK;
}

static void layout(sv_batch *b)
{
    auto &L = b->lay;
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        const uint64_t o = off;
        off = align_up(off + std::max<uint64_t>(bytes, 8), 256);
        return o;
    };
    const uint64_t S = (uint64_t)b->shots;
    L.prog = take((uint64_t)b->program_bytes);
    L.memory = take(S * 8);
    L.margins = take(S * 8);
    L.perm = take(S * 4);
    L.tmp = take(S * 4);
    L.waiting = take(S * 4);
    L.queue = take(S * sizeof(BranchRec));
    L.ready = take(S * 4);
    L.ctl = take(sizeof(Control));
    L.free_slots = take((uint64_t)std::max(b->slots, 1) * 4);
    const uint64_t n_tiles = b->resident ? 1 : (1ull << (b->n - b->tile_q));
    uint64_t ts = (uint64_t)b->workers * n_tiles * 8;
    if (b->mode == SV_MODE_PLAIN)  // partial sums, chunk sums and the decision cell
        ts = (uint64_t)kPlainRedBlocks * 17 * 8 + (((1ull << b->n) + 255) / 256) * 8 + 64;
    L.tile_sums = take(ts);
    L.dump = take(b->dump_shot >= 0 ? (16ull << b->n) : 8);
    L.counts_tmp = take(b->no_counts ? 8 : svb_counts_temp_bytes((int64_t)S));
    L.keys_sorted = take(b->no_counts ? 8 : S * 8);
    L.uniq = take(b->no_counts ? 8 : S * 8);
    L.cnt = take(b->no_counts ? 8 : S * 4);
    L.nuniq = take(8);
    L.slots = take((uint64_t)b->slots * state_bytes(b));
    L.total = off;
}

// ------------------------------------------------------------------ ops
struct XOp {  // expanded op
    int kind;       // sv_op_kind, or -1 Pauli channel, -2 Kraus channel
    int rule;
    int u3_index = -1;  // U3 ops: their index among the circuit's U3 ops
    uint64_t cond_mask = 0, cond_value = 0;  // condition (BFUNC: its predicate)
    std::vector<int> q, c;
    double p[3];
    std::vector<cd> mat;  // gates: dense matrix (row-major, bit t <-> q[t])
};

static bool is_gate_kind(uint32_t k)
{
    return (k >= SV_OP_ID && k <= SV_OP_TDG) || k == SV_OP_U3 || k == SV_OP_CX ||
           k == SV_OP_CZ || k == SV_OP_SWAP || k == SV_OP_UNITARY;
}
static int gate_nq(uint32_t k, uint32_t nq)
{
    if (k == SV_OP_CX || k == SV_OP_CZ || k == SV_OP_SWAP) return 2;
    if (k == SV_OP_UNITARY) return (int)nq;
    return 1;
}

// OpenQASM 2 U3 and the fixed one-qubit gates.
static std::vector<cd> gate_1q(uint32_t k, const double *p)
{
    const cd I(0, 1);
    const double h = 1.0 / std::sqrt(2.0);
    switch (k) {
    case SV_OP_ID: return {1, 0, 0, 1};
    case SV_OP_X: return {0, 1, 1, 0};
    case SV_OP_Y: return {0, -I, I, 0};
    case SV_OP_Z: return {1, 0, 0, -1};
    case SV_OP_H: return {h, h, h, -h};
    case SV_OP_S: return {1, 0, 0, I};
    case SV_OP_SDG: return {1, 0, 0, -I};
    case SV_OP_T: return {1, 0, 0, std::polar(1.0, M_PI / 4)};
    case SV_OP_TDG: return {1, 0, 0, std::polar(1.0, -M_PI / 4)};
    case SV_OP_U3: {
        const double c = std::cos(p[0] * 0.5), s = std::sin(p[0] * 0.5);
        return {c, -std::polar(s, p[2]), std::polar(s, p[1]), std::polar(c, p[1] + p[2])};
    }
    default: return {};
    }
}

struct Rule {
    bool kraus;
    int nq, n_terms;
    uint64_t mask;
    std::vector<double> prob;
    std::vector<uint8_t> codes;
    std::vector<std::vector<cd>> mats;
};

static sv_status validate_and_expand(const sv_batch *b, const sv_op *ops, size_t n_ops,
                                     const sv_noise_model *nm, std::vector<Rule> &rules,
                                     std::vector<XOp> &xo, double &ro01, double &ro10,
                                     uint64_t &gate_count)
{
    const int n = b->n;
    rules.clear();
    ro01 = ro10 = 0;
    if (nm) {
        if (nm->n_rules && !nm->rules) return fail(SV_EINVAL, "noise model: rules is NULL");
        ro01 = nm->readout_p01;
        ro10 = nm->readout_p10;
        if (!(ro01 >= 0 && ro01 <= 1 && ro10 >= 0 && ro10 <= 1))
            return fail(SV_EINVAL, "readout probabilities outside [0,1]");
        for (uint32_t r = 0; r < nm->n_rules; ++r) {
            const sv_noise_rule &nr = nm->rules[r];
            if (!nr.channel) return fail(SV_EINVAL, "rule %u: channel is NULL", r);
            Rule R;
            R.mask = nr.gate_kinds_mask;
            R.kraus = nr.is_kraus != 0;
            if (!R.kraus) {
                const auto *pc = (const sv_pauli_channel *)nr.channel;
                R.nq = (int)pc->nq;
                R.n_terms = (int)pc->n_terms;
                if (R.nq < 1 || R.nq > kMaxPauliQ) return fail(SV_EUNSUPPORTED, "rule %u: Pauli channel on %d qubits (1..%d)", r, R.nq, kMaxPauliQ);
                if (R.n_terms < 1 || R.n_terms > kMaxPauliTerms) return fail(SV_EINVAL, "rule %u: %d Pauli terms (1..%d)", r, R.n_terms, kMaxPauliTerms);
                if (!pc->prob || !pc->pauli) return fail(SV_EINVAL, "rule %u: NULL table", r);
                double sum = 0;
                for (int j = 0; j < R.n_terms; ++j) {
                    const double p = pc->prob[j];
                    if (!(p >= 0)) return fail(SV_EINVAL, "rule %u: negative probability", r);
                    R.prob.push_back(p);
                    sum += p;
                    for (int t = 0; t < R.nq; ++t) {
                        const uint8_t code = pc->pauli[j * R.nq + t];
                        if (code > 3) return fail(SV_EINVAL, "rule %u: Pauli code %u", r, code);
                        R.codes.push_back(code);
                    }
                }
                if (std::fabs(sum - 1.0) > 1e-12) return fail(SV_EINVAL, "rule %u: probabilities sum to %.17g", r, sum);
            } else {
                const auto *kc = (const sv_kraus_channel *)nr.channel;
                R.nq = (int)kc->nq;
                R.n_terms = (int)kc->n_mats;
                if (R.nq < 1 || R.nq > kMaxDenseQ) return fail(SV_EUNSUPPORTED, "rule %u: Kraus channel on %d qubits (1..%d)", r, R.nq, kMaxDenseQ);
                if (!kc->mats) return fail(SV_EINVAL, "rule %u: NULL matrices", r);
                if (R.n_terms < 1 || R.n_terms > kMaxKraus) return fail(SV_EUNSUPPORTED, "rule %u: %d Kraus matrices (1..%d)", r, R.n_terms, kMaxKraus);
                const int d = 1 << R.nq;
                std::vector<cd> sum(d * d, 0.0);
                for (int j = 0; j < R.n_terms; ++j) {
                    std::vector<cd> m(d * d);
                    for (int e = 0; e < d * d; ++e)
                        m[e] = cd(kc->mats[(size_t)(j * d * d + e) * 2], kc->mats[(size_t)(j * d * d + e) * 2 + 1]);
                    for (int a = 0; a < d; ++a)
                        for (int c = 0; c < d; ++c)
                            for (int x = 0; x < d; ++x) sum[a * d + c] += std::conj(m[x * d + a]) * m[x * d + c];
                    R.mats.push_back(m);
                }
                for (int a = 0; a < d; ++a)
                    for (int c = 0; c < d; ++c)
                        if (std::abs(sum[a * d + c] - (a == c ? 1.0 : 0.0)) > 1e-10)
                            return fail(SV_EINVAL, "rule %u: Kraus matrices are not complete", r);
            }
            rules.push_back(R);
        }
    }
    xo.clear();
    gate_count = 0;
    int n_u3 = 0;
    int terminal_seen = 0;
    for (size_t i = 0; i < n_ops; ++i) {
        const sv_op &op = ops[i];
        const uint32_t k = op.kind;
        const bool gate = is_gate_kind(k);
        const bool meas = k == SV_OP_MEASURE || k == SV_OP_RESET || k == SV_OP_MEASURE_RESET;
        if (op.cond_value & ~op.cond_mask)
            return fail(SV_EINVAL, "op %zu: condition value has bits outside its mask", i);
        if (k == SV_OP_BFUNC) {  // branch op: no qubits, one clbit
            if (op.nq != 0) return fail(SV_EINVAL, "op %zu: branch op takes no qubits", i);
            if (op.c[0] >= SV_MAX_CLBITS) return fail(SV_EINVAL, "op %zu: clbit %u >= 64", i, op.c[0]);
            XOp x;
            x.kind = (int)k;
            x.rule = -1;
            x.c.push_back((int)op.c[0]);
            x.cond_mask = op.cond_mask;
            x.cond_value = op.cond_value;
            x.p[0] = x.p[1] = x.p[2] = 0;
            xo.push_back(x);
            continue;
        }
        if (!gate && !meas) return fail(SV_EINVAL, "op %zu: unknown kind %u", i, k);
        const int nq = gate ? gate_nq(k, op.nq) : (int)op.nq;
        if (gate && k != SV_OP_UNITARY && op.nq != (uint32_t)nq && op.nq != 0)
            return fail(SV_EINVAL, "op %zu: kind %u acts on %d qubits, nq=%u", i, k, nq, op.nq);
        if (nq < 1) return fail(SV_EINVAL, "op %zu: no qubits", i);
        if (k == SV_OP_UNITARY && (nq > kMaxDenseQ || !op.mat))
            return fail(nq > kMaxDenseQ ? SV_EUNSUPPORTED : SV_EINVAL,
                        "op %zu: unitary on %d qubits (1..%d, mat required)", i, nq, kMaxDenseQ);
        const uint32_t *qs = nq > SV_MAX_INLINE ? op.q_ext : op.q;
        const uint32_t *cs = nq > SV_MAX_INLINE ? op.c_ext : op.c;
        if (!qs) return fail(SV_EINVAL, "op %zu: qubit list is NULL", i);
        XOp x;
        x.kind = (int)k;
        x.rule = -1;
        if (k == SV_OP_U3) x.u3_index = n_u3++;
        x.cond_mask = op.cond_mask;
        x.cond_value = op.cond_value;
        uint64_t seen = 0;
        for (int t = 0; t < nq; ++t) {
            if (qs[t] >= (uint32_t)n) return fail(SV_EINVAL, "op %zu: qubit %u out of range", i, qs[t]);
            if (seen >> qs[t] & 1) return fail(SV_EINVAL, "op %zu: repeated qubit %u", i, qs[t]);
            seen |= 1ull << qs[t];
            x.q.push_back((int)qs[t]);
        }
        if (k == SV_OP_MEASURE || k == SV_OP_MEASURE_RESET) {
            if (!cs) return fail(SV_EINVAL, "op %zu: clbit list is NULL", i);
            for (int t = 0; t < nq; ++t) {
                if (cs[t] >= SV_MAX_CLBITS) return fail(SV_EINVAL, "op %zu: clbit %u >= 64", i, cs[t]);
                x.c.push_back((int)cs[t]);
            }
        }
        std::memcpy(x.p, op.p, sizeof x.p);
        if (gate) {
            ++gate_count;
            if (k == SV_OP_CX || k == SV_OP_CZ || k == SV_OP_SWAP) {
            } else if (k == SV_OP_UNITARY) {
                const int d = 1 << nq;
                x.mat.resize(d * d);
                for (int e = 0; e < d * d; ++e) x.mat[e] = cd(op.mat[2 * e], op.mat[2 * e + 1]);
                for (int a = 0; a < d; ++a)
                    for (int c = 0; c < d; ++c) {
                        cd s = 0;
                        for (int y = 0; y < d; ++y) s += std::conj(x.mat[y * d + a]) * x.mat[y * d + c];
                        if (std::abs(s - (a == c ? 1.0 : 0.0)) > 1e-10)
                            return fail(SV_EINVAL, "op %zu: matrix is not unitary", i);
                    }
            } else {
                x.mat = gate_1q(k, op.p);
            }
        }
        xo.push_back(x);
        if (gate) {
            for (size_t r = 0; r < rules.size(); ++r) {
                if (k >= 64 || !((rules[r].mask >> k) & 1)) continue;
                if (rules[r].nq != nq) continue;  // a rule attaches to gates of its own width only
                XOp ch;
                ch.kind = rules[r].kraus ? -2 : -1;
                ch.rule = (int)r;
                ch.q = x.q;
                ch.cond_mask = x.cond_mask;  // noise of a conditional gate is conditional too
                ch.cond_value = x.cond_value;
                xo.push_back(ch);
            }
        }
        (void)terminal_seen;
    }
    if (xo.size() > 0x7fffffff) return fail(SV_EINVAL, "too many ops");
    return SV_OK;
}

// ------------------------------------------------------------------ planner
// Ops may be executed in any order that keeps (a) the order of ops sharing a
// qubit and (b) the relative order of the state-dependent random ops (Kraus
// channels, measure, reset). Unitaries and drawn Pauli strings on other
// qubits commute with a Kraus or measure op and do not change its outcome
// probabilities, so every per-shot decision is unchanged by such a reorder.
//
// Passes: greedy in list order, an op joins the current pass if all its
// predecessors are already placed and its qubits fit in the k tile qubits
// (which always include qubits 0..3, so global accesses are 128-byte runs).
// Groups: the same greedy inside a pass with r = log2(amplitudes per
// thread) register bits. Measures and dense 4x4 ops form groups of their own
// that run as LDS sweeps. The final measurement of all qubits gets a pass of
// its own with tile qubits 0..k-1 (contiguous chunks for sampling).


// Ops whose effect depends on, or changes, per-shot state beyond their qubits:
// Kraus channels and measurements (outcome probabilities), conditional ops
// and branch ops (the classical register).
static bool op_ordered(const XOp &x)
{
    return x.kind == -2 || x.kind == SV_OP_MEASURE || x.kind == SV_OP_RESET ||
           x.kind == SV_OP_MEASURE_RESET || x.kind == SV_OP_BFUNC || x.cond_mask != 0;
}

// Ops that run as LDS sweeps rather than in register groups: measurements,
// dense matrices on two or more qubits (unitaries, Kraus channels), and
// Pauli channels on more qubits than a register group holds (r).
static bool op_fallback(const XOp &x, const std::vector<Rule> &rules, int r)
{
    if (x.kind == SV_OP_MEASURE || x.kind == SV_OP_RESET || x.kind == SV_OP_MEASURE_RESET) return true;
    if (x.kind == SV_OP_UNITARY && x.q.size() >= 2) return true;
    if (x.kind == -2 && rules[x.rule].nq >= 2) return true;
    if (x.kind == -1 && rules[x.rule].nq > r) return true;
    return false;
}

static uint32_t qmask_of(const XOp &x)
{
    uint32_t m = 0;
    for (int q : x.q) m |= 1u << q;
    return m;
}

// effect of tile bit b on the low six bits of its swizzled LDS position
// (the executor's swizzle adds bits 6+j and 7+j to bit j, for j in swz)
static uint32_t fold_vec(int b, uint32_t swz)
{
    if (b < 6) return 1u << b;
    const uint32_t i = 1u << b;
    return ((i >> 6) ^ (i >> 7)) & swz & 63u;
}

static int gf2_rank_add(uint32_t basis[6], uint32_t v)
{
    for (int i = 5; i >= 0; --i) {
        if (!((v >> i) & 1)) continue;
        if (!basis[i]) {
            basis[i] = v;
            return 1;
        }
        v ^= basis[i];
    }
    return 0;
}

// A gate and the channel ops the noise model attached to it (they follow it
// in the expanded list, on a subset of its qubits) are placed as one unit:
// taking a gate into a pass or group while deferring its channel would
// split the fused one-qubit factor of that qubit into two micro-ops.
static size_t unit_end(const std::vector<XOp> &xo, const std::vector<uint32_t> &list, size_t idx,
                       const std::vector<Rule> &rules, bool groups, int r)
{
    const XOp &g = xo[list[idx]];
    size_t e = idx + 1;
    if (g.kind < 0 || !is_gate_kind((uint32_t)g.kind) || (groups && op_fallback(g, rules, r))) return e;
    const uint32_t m = qmask_of(g);
    while (e < list.size() && list[e] == list[e - 1] + 1) {
        const XOp &x = xo[list[e]];
        if (x.kind >= 0 || (qmask_of(x) & ~m) || (groups && op_fallback(x, rules, r))) break;
        ++e;
    }
    return e;
}

// Tile sets tried per pass of a streamed state, besides the greedy one, and
// rounds of single-qubit exchanges from the best of them. The search is
// bounded for large circuits: each candidate looks at most kSearchUnits
// units ahead, and circuits of more than kSearchMaxOps expanded ops keep
// the greedy sets (host planning stays well under a second)
constexpr int kPassCandidates = 200;
constexpr int kPassExchangeRounds = 4;
constexpr size_t kSearchUnits = 4096;
constexpr size_t kSearchMaxOps = 32768;

static void plan_program(int n, int k, int r, bool resident, bool use_groups, uint32_t swz, int span,
                         const std::vector<XOp> &xo, const std::vector<Rule> &rules,
                         bool terminal, Plan &P)
{
    P = Plan();
    const uint32_t N = (uint32_t)xo.size();
    const uint32_t body = terminal ? N - 1 : N;
    const uint32_t all = (n >= 32) ? 0xffffffffu : ((1u << n) - 1);
    const uint32_t base_mask = resident ? all : ((1u << kCoalesceQ) - 1);
    std::vector<uint32_t> remaining(body);
    for (uint32_t j = 0; j < body; ++j) remaining[j] = j;

    auto emit_pass = [&](const std::vector<uint32_t> &sel, uint32_t tmask) {
        for (int q = 0; q < n && __builtin_popcount(tmask) < k; ++q) tmask |= 1u << q;
        PassInfo pi;
        std::memset(&pi, 0, sizeof pi);
        pi.first_op = (uint32_t)P.order.size();
        pi.tmask = tmask;
        int a = 0, g = 0, lbit[32];
        for (int q = 0; q < n; ++q) {
            if ((tmask >> q) & 1) {
                lbit[q] = a;
                pi.tq[a++] = (uint8_t)q;
            } else {
                lbit[q] = -1;
                pi.gq[g++] = (uint8_t)q;
            }
        }
        pi.contiguous = (tmask == (k >= 32 ? 0xffffffffu : ((1u << k) - 1)));
        const uint32_t pidx = (uint32_t)P.passes.size();
        // groups inside the pass
        std::vector<uint32_t> grem = sel;
        while (!grem.empty()) {
            std::vector<uint32_t> gsel, grest;
            uint32_t G = 0, blocked = 0;
            bool ord_blocked = false, fb_group = false;
            for (size_t idx = 0; idx < grem.size();) {
                const uint32_t j = grem[idx];
                const XOp &x = xo[j];
                const bool fb = !use_groups || op_fallback(x, rules, r);
                if (fb) {
                    const uint32_t m = qmask_of(x);
                    const bool ord = op_ordered(x);
                    const bool ok = !(m & blocked) && !(ord && ord_blocked);
                    if (ok && gsel.empty()) {
                        gsel.push_back(j);
                        fb_group = true;
                        for (size_t t = idx + 1; t < grem.size(); ++t) grest.push_back(grem[t]);
                        break;
                    }
                    blocked |= m;
                    ord_blocked |= ord;
                    grest.push_back(j);
                    ++idx;
                    continue;
                }
                const size_t e = unit_end(xo, grem, idx, rules, true, r);
                uint32_t m = 0;
                bool ord = false;
                for (size_t t = idx; t < e; ++t) {
                    m |= qmask_of(xo[grem[t]]);
                    ord = ord || op_ordered(xo[grem[t]]);
                }
                const bool ok = !(m & blocked) && !(ord && ord_blocked) &&
                                __builtin_popcount(G | m) <= r;
                for (size_t t = idx; t < e; ++t) (ok ? gsel : grest).push_back(grem[t]);
                if (ok) {
                    G |= m;
                } else {
                    blocked |= m;
                    ord_blocked |= ord;
                }
                idx = e;
            }
            GroupInfo gi;
            std::memset(&gi, 0, sizeof gi);
            gi.first_op = (uint32_t)P.order.size();
            gi.fallback = fb_group ? 1u : 0u;
            if (!fb_group && use_groups) {
                // register bits: the group's tile bits, then padding. Lanes:
                // the lanes that one LDS cycle serves hit distinct banks when
                // their thread bits map to independent vectors in the low
                // bits of the swizzled amplitude index. Measured on gfx950
                // for 8-byte accesses: a write cycle serves 16 lanes (thread
                // bits 0..3 should span index bits 0..3), a read cycle 32
                // (thread bits 0..4, index bits 0..4). So thread bits
                // 0..span-2 are chosen first, then bit span-1; taking
                // independent vectors greedily reaches the largest rank at
                // each stage (a matroid). The other thread bits take what
                // is left
                uint32_t reg_tile = 0;
                for (int q = 0; q < n; ++q)
                    if ((G >> q) & 1) reg_tile |= 1u << lbit[q];
                std::vector<int> cand;
                for (int b = 0; b < k; ++b)
                    if (!((reg_tile >> b) & 1)) cand.push_back(b);
                std::vector<int> lanes, others;
                uint32_t taken = 0;
                for (int want = span - 1; want <= span; ++want) {
                    const uint32_t low = (1u << want) - 1u;
                    uint32_t basis[6] = {0, 0, 0, 0, 0, 0};
                    for (int b : lanes) gf2_rank_add(basis, fold_vec(b, swz) & low);
                    for (int b : cand) {
                        if ((int)lanes.size() >= want) break;
                        if (!((taken >> b) & 1u) && gf2_rank_add(basis, fold_vec(b, swz) & low)) {
                            lanes.push_back(b);
                            taken |= 1u << b;
                        }
                    }
                }
                for (int b : cand)
                    if (!((taken >> b) & 1u)) others.push_back(b);
                // padding of the register bits comes from bits not used as lanes
                std::vector<int> regs;
                for (int b = 0; b < k; ++b)
                    if ((reg_tile >> b) & 1) regs.push_back(b);
                std::vector<int> rest2;
                for (int b : others) {
                    if ((int)regs.size() < r) regs.push_back(b);
                    else rest2.push_back(b);
                }
                while ((int)lanes.size() < 6 && !rest2.empty()) {
                    lanes.push_back(rest2.front());
                    rest2.erase(rest2.begin());
                }
                std::sort(regs.begin(), regs.end());
                for (int j = 0; j < r; ++j) gi.gpos[j] = (uint8_t)regs[j];
                int ci = 0;
                for (int b : lanes) gi.cpos[ci++] = (uint8_t)b;
                for (int b : rest2) gi.cpos[ci++] = (uint8_t)b;
            }
            const uint32_t gidx = (uint32_t)P.groups.size();
            for (uint32_t j : gsel) {
                P.order.push_back(j);
                P.op_pass.push_back(pidx);
                P.op_group.push_back(gidx);
            }
            gi.end_op = (uint32_t)P.order.size();
            P.groups.push_back(gi);
            grem.swap(grest);
        }
        pi.end_op = (uint32_t)P.order.size();
        P.passes.push_back(pi);
    };

    // One pass over the remaining ops, in list order: a unit (a gate and its
    // channels) is taken when no earlier deferred unit shares a qubit with
    // it (nor, for ordered ops, comes before it) and it fits the tile set.
    // With fixed == 0 the tile set grows from base_mask as units are taken
    // (greedy); otherwise it is `fixed`.
    auto take = [&](uint32_t fixed, std::vector<uint32_t> &sel, std::vector<uint32_t> &rest) {
        sel.clear();
        rest.clear();
        uint32_t T = fixed ? fixed : base_mask, blocked = 0;
        bool ord_blocked = false;
        for (size_t idx = 0; idx < remaining.size();) {
            const size_t e = unit_end(xo, remaining, idx, rules, false, r);
            if (sel.size() + (e - idx) > (size_t)kMaxPassOps) {
                rest.insert(rest.end(), remaining.begin() + idx, remaining.end());
                break;
            }
            uint32_t m = 0;
            bool ord = false;
            for (size_t t = idx; t < e; ++t) {
                m |= qmask_of(xo[remaining[t]]);
                ord = ord || op_ordered(xo[remaining[t]]);
            }
            const bool fits = fixed ? !(m & ~fixed) : __builtin_popcount(T | m) <= k;
            const bool ok = !(m & blocked) && !(ord && ord_blocked) && fits;
            for (size_t t = idx; t < e; ++t) (ok ? sel : rest).push_back(remaining[t]);
            if (ok) {
                T |= m;
            } else {
                blocked |= m;
                ord_blocked |= ord;
            }
            idx = e;
        }
        return T;
    };
    // Streamed states: besides the greedy tile set, try fixed sets made of
    // the qubits in order of first use among the next units, and seeded
    // perturbations of that order, and keep the set that takes the most
    // ops (fewer passes over the state). Deterministic for a circuit.
    const bool search = !resident && n > k && xo.size() <= kSearchMaxOps;
    uint64_t rng = 0x9e3779b97f4a7c15ull;
    auto next_rand = [&rng]() {
        // splitmix64
        uint64_t z = (rng += 0x9e3779b97f4a7c15ull);
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        return z ^ (z >> 31);
    };
    std::vector<uint32_t> um, ulen;   // units of the remaining list: qubit mask, op count
    std::vector<uint8_t> uord;        // unit holds an ordered op
    auto count_fixed = [&](uint32_t C) {
        uint32_t blocked = 0;
        bool ord_blocked = false;
        size_t taken = 0;
        for (size_t u = 0; u < um.size() && u < kSearchUnits; ++u) {
            if (taken + ulen[u] > (size_t)kMaxPassOps) break;
            if (!(um[u] & blocked) && !(uord[u] && ord_blocked) && !(um[u] & ~C)) {
                taken += ulen[u];
            } else {
                blocked |= um[u];
                ord_blocked = ord_blocked || uord[u];
            }
        }
        return taken;
    };
    while (!remaining.empty()) {
        std::vector<uint32_t> sel, rest;
        uint32_t T = take(0, sel, rest);
        if (search && !rest.empty()) {
            um.clear();
            ulen.clear();
            uord.clear();
            for (size_t idx = 0; idx < remaining.size();) {
                const size_t e = unit_end(xo, remaining, idx, rules, false, r);
                uint32_t m = 0;
                bool ord = false;
                for (size_t t = idx; t < e; ++t) {
                    m |= qmask_of(xo[remaining[t]]);
                    ord = ord || op_ordered(xo[remaining[t]]);
                }
                um.push_back(m);
                ulen.push_back((uint32_t)(e - idx));
                uord.push_back(ord ? 1 : 0);
                idx = e;
            }
            std::vector<int> order;
            uint32_t seen = base_mask;
            for (size_t u = 0; u < um.size() && u < 256; ++u)
                for (int q = 0; q < n; ++q)
                    if (((um[u] & ~seen) >> q) & 1u) {
                        order.push_back(q);
                        seen |= 1u << q;
                    }
            for (int q = 0; q < n; ++q)
                if (!((seen >> q) & 1u)) order.push_back(q);
            const int free_q = k - __builtin_popcount(base_mask);
            size_t best = sel.size();
            uint32_t best_c = 0;
            for (int cand = 0; cand <= kPassCandidates; ++cand) {
                std::vector<int> o2 = order;
                if (cand > 0) {
                    const int swaps = (int)(next_rand() % 5);
                    for (int t = 0; t < swaps; ++t) {
                        const size_t i = next_rand() % o2.size(), j = next_rand() % o2.size();
                        std::swap(o2[i], o2[j]);
                    }
                }
                uint32_t C = base_mask;
                for (int t = 0; t < free_q && t < (int)o2.size(); ++t) C |= 1u << o2[t];
                const size_t got = count_fixed(C);
                if (got > best) {
                    best = got;
                    best_c = C;
                }
            }
            // then exchange one tile qubit for one outside while that helps
            for (int round = 0; round < kPassExchangeRounds && best_c; ++round) {
                uint32_t step_c = 0;
                size_t step_best = best;
                for (int a = 0; a < n; ++a) {
                    if (!((best_c >> a) & 1u) || ((base_mask >> a) & 1u)) continue;
                    for (int q = 0; q < n; ++q) {
                        if ((best_c >> q) & 1u) continue;
                        const uint32_t C = (best_c & ~(1u << a)) | (1u << q);
                        const size_t got = count_fixed(C);
                        if (got > step_best) {
                            step_best = got;
                            step_c = C;
                        }
                    }
                }
                if (!step_c) break;
                best = step_best;
                best_c = step_c;
            }
            if (best_c) T = take(best_c, sel, rest);
        }
        emit_pass(sel, T);
        remaining.swap(rest);
    }
    if (terminal) {
        // final measure-all: one op, contiguous tiles, its own fallback group
        PassInfo pi;
        std::memset(&pi, 0, sizeof pi);
        pi.first_op = (uint32_t)P.order.size();
        const uint32_t tm = resident ? all : ((1u << k) - 1);
        pi.tmask = tm;
        int a = 0, g = 0;
        for (int q = 0; q < n; ++q) {
            if ((tm >> q) & 1) pi.tq[a++] = (uint8_t)q;
            else pi.gq[g++] = (uint8_t)q;
        }
        pi.contiguous = 1;
        GroupInfo gi;
        std::memset(&gi, 0, sizeof gi);
        gi.first_op = pi.first_op;
        gi.fallback = 1;
        P.order.push_back(N - 1);
        P.op_pass.push_back((uint32_t)P.passes.size());
        P.op_group.push_back((uint32_t)P.groups.size());
        gi.end_op = (uint32_t)P.order.size();
        P.groups.push_back(gi);
        pi.end_op = (uint32_t)P.order.size();
        P.passes.push_back(pi);
    }
}

static void rule_dev(const Rule &R, std::vector<double> &pool, DevRule &d)
{
    std::memset(&d, 0, sizeof d);
    d.is_kraus = R.kraus;
    d.nq = (uint32_t)R.nq;
    d.n_terms = (uint32_t)R.n_terms;
    if (!R.kraus) {
        d.thr = (uint32_t)pool.size();
        double run = 0;
        for (int j = 0; j < R.n_terms; ++j) {  // running sums in list order
            run += R.prob[j];
            pool.push_back(run);
        }
        // term codes x | z << 8 | ny << 16, one double each (exact integers)
        d.codes = (uint32_t)pool.size();
        for (int j = 0; j < R.n_terms; ++j) {
            uint32_t x = 0, z = 0, ny = 0;
            for (int t = 0; t < R.nq; ++t) {
                const uint8_t c = R.codes[j * R.nq + t];
                if (c == 1 || c == 2) x |= 1u << t;
                if (c == 3 || c == 2) z |= 1u << t;
                if (c == 2) ++ny;
            }
            pool.push_back((double)(x | (z << 8) | (ny << 16)));
        }
    } else {
        d.mats = (uint32_t)pool.size();
        const int dd = 1 << R.nq;
        for (const auto &m : R.mats)
            for (const cd &v : m) {
                pool.push_back(v.real());
                pool.push_back(v.imag());
            }
        // K^dagger K diagonal? smallest eigenvalue of K0^dagger K0
        bool diag = true;
        std::vector<cd> M0(dd * dd);
        for (size_t j = 0; j < R.mats.size(); ++j) {
            const auto &m = R.mats[j];
            for (int a = 0; a < dd; ++a)
                for (int c = 0; c < dd; ++c) {
                    cd s = 0;
                    for (int x = 0; x < dd; ++x) s += std::conj(m[x * dd + a]) * m[x * dd + c];
                    if (a != c && std::abs(s) > 0) diag = false;
                    if (j == 0) M0[a * dd + c] = s;
                }
        }
        d.diag_mm = diag;
        // matrices that are c * I: choosing one leaves the state's direction
        // unchanged (only its norm), which every later decision divides out
        for (size_t j = 0; j < R.mats.size(); ++j) {
            const auto &m = R.mats[j];
            bool sc = true;
            for (int a = 0; a < dd && sc; ++a)
                for (int c = 0; c < dd && sc; ++c)
                    sc = (a == c) ? (m[a * dd + c] == m[0]) : (m[a * dd + c] == cd(0, 0));
            if (sc) d.scalar_mask |= 1u << j;
        }
        double lam;
        if (dd == 2) {
            const double a = M0[0].real(), c = M0[3].real();
            const double bb = std::norm(M0[1]);
            lam = 0.5 * (a + c) - std::sqrt(0.25 * (a - c) * (a - c) + bb);
        } else if (diag) {
            lam = M0[0].real();
            for (int a = 1; a < dd; ++a) lam = std::min(lam, M0[a * dd + a].real());
        } else {
            // Gershgorin lower bound (a valid lower bound of the eigenvalues)
            lam = 1e300;
            for (int a = 0; a < dd; ++a) {
                double rad = 0;
                for (int c = 0; c < dd; ++c)
                    if (c != a) rad += std::abs(M0[a * dd + c]);
                lam = std::min(lam, M0[a * dd + a].real() - rad);
            }
        }
        // keep a safety margin below the bound so that rounding in the state
        // reduction can never make K0 the wrong choice
        lam = lam * (1.0 - 1e-12) - 1e-15;
        d.lam_min0 = lam > 0 ? lam : 0.0;
    }
}

// ------------------------------------------------------------------ ABI
extern "C" {

const char *sv_last_error(void) { return g_err.c_str(); }

sv_status sv_batch_create(int n_qubits, int64_t n_shots, sv_dtype dtype, sv_batch **out)
{
    if (!out) return fail(SV_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_qubits < 1 || n_qubits > 30) return fail(SV_EINVAL, "n_qubits %d outside 1..30", n_qubits);
    if (n_shots < 1 || n_shots > 0x7fffffffLL) return fail(SV_EINVAL, "n_shots %lld outside 1..2^31-1", (long long)n_shots);
    if (dtype != SV_C64 && dtype != SV_C128) return fail(SV_EINVAL, "bad dtype %d", (int)dtype);
    sv_batch *b = new sv_batch;
    b->n = n_qubits;
    b->shots = n_shots;
    b->dtype = dtype;
    *out = b;
    return SV_OK;
}

sv_status sv_batch_set_option(sv_batch *b, const char *key, int64_t v)
{
    if (!b || !key) return fail(SV_EINVAL, "NULL argument");
    const std::string k = key;
    const bool sizing = k == "mode" || k == "slots" || k == "workers" || k == "tile_qubits" ||
                        k == "program_bytes" || k == "dump_shot" || k == "engine" ||
                        k == "pipeline";
    if (sizing && b->attached) return fail(SV_ESTATE, "option %s must be set before attach", key);
    if (sizing) b->auto_slots = b->auto_workers = 0;
    if (k == "mode") {
        if (v < 0 || v > 2) return fail(SV_EINVAL, "mode %lld", (long long)v);
        b->mode = (int)v;
    } else if (k == "slots") {
        if (v < 0 || v > (1 << 24)) return fail(SV_EINVAL, "slots %lld", (long long)v);
        b->opt_slots = v;
    } else if (k == "workers") {
        if (v < 0 || v > (1 << 20)) return fail(SV_EINVAL, "workers %lld", (long long)v);
        b->opt_workers = v;
    } else if (k == "tile_qubits") {
        if (v != 0 && (v < 6 || v > kMaxTileQ)) return fail(SV_EINVAL, "tile_qubits %lld (0 or 6..14)", (long long)v);
        b->opt_tile = v;
    } else if (k == "program_bytes") {
        if (v < 4096) return fail(SV_EINVAL, "program_bytes %lld", (long long)v);
        b->program_bytes = v;
    } else if (k == "dump_shot") {
        if (v < -1 || v >= b->shots) return fail(SV_EINVAL, "dump_shot %lld", (long long)v);
        b->dump_shot = v;
    } else if (k == "engine") {
        if (v < 0 || v > 2)
            return fail(SV_EINVAL, "engine %lld (0 automatic, 1 LDS sweeps, 2 register groups)", (long long)v);
        b->opt_engine = v;
    } else if (k == "pipeline") {
        if (v < -1 || v > 1) return fail(SV_EINVAL, "pipeline %lld (-1 automatic, 0, 1)", (long long)v);
        b->opt_pipeline = v;
    } else if (k == "mfma") {
        if (v < 0 || v > 2)
            return fail(SV_EINVAL, "mfma %lld (0 automatic, 1 vector ALU, 2 matrix cores)", (long long)v);
        b->opt_mfma = v;
    } else if (k == "graph") {
        if (v < 0 || v > 1) return fail(SV_EINVAL, "graph %lld (0 or 1)", (long long)v);
        b->opt_graph = v;
    } else if (k == "shot_offset") {
        if (v < 0) return fail(SV_EINVAL, "shot_offset %lld", (long long)v);
        b->shot_offset = v;
    } else if (k == "spin_limit_ms") {
        if (v < 1) return fail(SV_EINVAL, "spin_limit_ms %lld", (long long)v);
        b->spin_ms = v;
    } else if (k == "spin_elapsed") {
        if (v < 0 || v > 1) return fail(SV_EINVAL, "spin_elapsed %lld (0 or 1)", (long long)v);
        b->spin_elapsed = v;
    } else {
        return fail(SV_EINVAL, "unknown option '%s'", key);
    }
    return SV_OK;
}

sv_status sv_batch_footprint(const sv_batch *cb, uint64_t *bytes_required, uint64_t *bytes_per_state)
{
    if (!cb) return fail(SV_EINVAL, "NULL handle");
    sv_batch *b = const_cast<sv_batch *>(cb);
    sv_status s = derive(b);
    if (s != SV_OK) return s;
    layout(b);
    if (bytes_required) *bytes_required = b->lay.total;
    if (bytes_per_state) *bytes_per_state = state_bytes(b);
    return SV_OK;
}

sv_status sv_batch_attach(sv_batch *b, void *arena, uint64_t bytes, void *stream)
{
    if (!b || !arena) return fail(SV_EINVAL, "NULL argument");
    if (((uintptr_t)arena & 255) != 0) return fail(SV_EINVAL, "arena must be 256-byte aligned");
    sv_status s = derive(b);
    if (s != SV_OK) return s;
    layout(b);
    if (bytes < b->lay.total)
        return fail(SV_ENOMEM, "arena holds %llu bytes, %llu required",
                    (unsigned long long)bytes, (unsigned long long)b->lay.total);
    b->arena = (char *)arena;
    b->arena_bytes = bytes;
    b->stream = (hipStream_t)stream;
    if (!b->ev0) {
        HIPCHK(hipEventCreate(&b->ev0));
        HIPCHK(hipEventCreate(&b->ev1));
        HIPCHK(hipEventCreate(&b->ev2));
        HIPCHK(hipEventCreate(&b->ev3));
    }
    b->attached = true;
    b->have_results = false;
    return SV_OK;
}

// A circuit without ops: every shot keeps the all-zero register and the
// state stays |0..0>. Only the initialisation kernel runs (it clears the
// per-shot registers); a requested state dump is written as |0..0>.
static sv_status run_empty(sv_batch *b)
{
    char *A = b->arena;
    const auto &L = b->lay;
    ExecParams P;
    std::memset(&P, 0, sizeof P);
    P.memory = (uint64_t *)(A + L.memory);
    P.margins = (uint64_t *)(A + L.margins);
    P.shot_perm = (int32_t *)(A + L.perm);
    P.queue = (BranchRec *)(A + L.queue);
    P.ready = (uint32_t *)(A + L.ready);
    P.ctl = (Control *)(A + L.ctl);
    P.free_slots = (int32_t *)(A + L.free_slots);
    P.n_shots = b->shots;
    P.queue_cap = (int32_t)b->shots;
    HIPCHK(ev_record(b->ev0, b->stream));
    HIPCHK(svb_launch_init(&P, 0, (int)b->shots, -1, 0, b->stream));
    if (b->dump_shot >= 0) {
        static const double one = 1.0;
        HIPCHK(hipMemsetAsync(A + L.dump, 0, 16ull << b->n, b->stream));
        HIPCHK(hipMemcpyAsync(A + L.dump, &one, sizeof one, hipMemcpyHostToDevice, b->stream));
    }
    HIPCHK(ev_record(b->ev1, b->stream));
    HIPCHK(ev_wait(b->ev1, b->stream));
    float ms = 0;
    HIPCHK(ev_ms(&ms, b->ev0, b->ev1));
    sv_stats &st = b->stats;
    std::memset(&st, 0, sizeof st);
    st.kernel_ms = ms;
    st.workers = (uint32_t)b->workers;
    st.slots = (uint32_t)b->slots;
    st.tile_qubits = (uint32_t)b->tile_q;
    st.tile_buffers = (uint32_t)b->nbuf;
    b->have_results = true;
    b->have_stats = true;
    b->have_dump = b->dump_shot >= 0;
    return SV_OK;
}

// FNV-1a hash of the op program (graph runs skip an unchanged upload)
static uint64_t blob_hash(const std::vector<char> &v)
{
    uint64_t h = 1469598103934665603ull;
    for (char ch : v) h = (h ^ (uint8_t)ch) * 1099511628211ull;
    return h ? h : 1;
}

static void graph_drop(sv_batch *b)
{
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->gexec = nullptr;
    b->graph = nullptr;
    b->n_init = b->n_exec = nullptr;
    b->graph_fn = nullptr;
}

// The run's initialisation and first executor launch as the handle's HIP
// graph: built once per executor instantiation, grid and LDS size; later
// runs only update the two kernel nodes' arguments, then replay it.
static sv_status graph_run(sv_batch *b, const ExecParams &P, int root_slot, int n_free)
{
    void *init_fn = nullptr, *exec_fn = nullptr;
    unsigned ig = 0, eg = 0, blk = 0;
    size_t lds = 0;
    HIPCHK(svb_graph_nodes(&P, b->dtype == SV_C128, b->reg_bits, b->workers, &init_fn, &ig, &exec_fn,
                           &eg, &blk, &lds));
    ExecParams Pc = P;
    int restart = 0, n_root = (int)b->shots, rs = root_slot, nf = n_free;
    void *iargs[] = {&Pc, &restart, &n_root, &rs, &nf};
    void *eargs[] = {&Pc};
    hipKernelNodeParams ip;
    std::memset(&ip, 0, sizeof ip);
    ip.func = init_fn;
    ip.gridDim = dim3(ig);
    ip.blockDim = dim3(blk);
    ip.sharedMemBytes = 0;
    ip.kernelParams = iargs;
    ip.extra = nullptr;
    hipKernelNodeParams ep;
    std::memset(&ep, 0, sizeof ep);
    ep.func = exec_fn;
    ep.gridDim = dim3(eg);
    ep.blockDim = dim3(blk);
    ep.sharedMemBytes = (unsigned)lds;
    ep.kernelParams = eargs;
    ep.extra = nullptr;
    if (b->gexec && b->graph_fn == exec_fn && b->graph_grid == eg && b->graph_lds == lds) {
        HIPCHK(hipGraphExecKernelNodeSetParams(b->gexec, b->n_init, &ip));
        HIPCHK(hipGraphExecKernelNodeSetParams(b->gexec, b->n_exec, &ep));
    } else {
        graph_drop(b);
        HIPCHK(hipGraphCreate(&b->graph, 0));
        HIPCHK(hipGraphAddKernelNode(&b->n_init, b->graph, nullptr, 0, &ip));
        HIPCHK(hipGraphAddKernelNode(&b->n_exec, b->graph, &b->n_init, 1, &ep));
        HIPCHK(hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0));
        b->graph_fn = exec_fn;
        b->graph_grid = eg;
        b->graph_lds = lds;
    }
    HIPCHK(hipGraphLaunch(b->gexec, b->stream));
    return SV_OK;
}

static sv_status run_impl(sv_batch *b, const sv_op *ops, size_t n_ops, const sv_noise_model *nm,
                          uint64_t seed, const double *params, size_t n_sets)
{
    if (!b) return fail(SV_EINVAL, "NULL handle");
    if (!ops && n_ops) return fail(SV_EINVAL, "ops is NULL");
    const bool sweep = params != nullptr;
    if (sweep) {
        if (b->mode != SV_MODE_BATCH) return fail(SV_EUNSUPPORTED, "parameter sweeps run in batch mode");
        if (n_sets == 0 || b->shots % (int64_t)n_sets != 0)
            return fail(SV_EINVAL, "n_sets %zu must divide the %lld shots", n_sets, (long long)b->shots);
        if ((uint64_t)b->shots / n_sets > 0xffffffffull) return fail(SV_EINVAL, "too many shots per set");
    }
    b->have_results = false;
    b->have_stats = false;
    b->have_dump = false;
    std::vector<Rule> rules;
    std::vector<XOp> xo;
    double ro01, ro10;
    uint64_t gate_count;
    sv_status s = validate_and_expand(b, ops, n_ops, nm, rules, xo, ro01, ro10, gate_count);
    if (s != SV_OK) return s;
    if (xo.empty()) {
        if (!b->attached) return fail(SV_ESTATE, "no arena attached");
        return run_empty(b);
    }

    const int n = b->n;
    // terminal measurement: last op measures every qubit in order
    bool terminal = false;
    {
        const XOp &last = xo.back();
        if (last.kind == SV_OP_MEASURE && (int)last.q.size() == n) {
            terminal = true;
            for (int t = 0; t < n; ++t) terminal = terminal && last.q[t] == t;
            terminal = terminal && last.cond_mask == 0;
        }
    }
    for (size_t j = 0; j < xo.size(); ++j) {
        const XOp &x = xo[j];
        const bool is_meas = x.kind == SV_OP_MEASURE || x.kind == SV_OP_RESET || x.kind == SV_OP_MEASURE_RESET;
        if (is_meas && !(terminal && j + 1 == xo.size()) && (int)x.q.size() > kMaxMeasQ)
            return fail(SV_EUNSUPPORTED, "measure of %zu qubits (at most %d unless it is a final measure of all qubits in order)",
                        x.q.size(), kMaxMeasQ);
    }
    if (!b->attached) return fail(SV_ESTATE, "no arena attached");
    // a streamed tile holds qubits 0..3 and the op's qubits
    if (!b->resident && b->mode != SV_MODE_PLAIN) {
        for (size_t j = 0; j < xo.size(); ++j) {
            const XOp &x = xo[j];
            const bool is_meas = x.kind == SV_OP_MEASURE || x.kind == SV_OP_RESET || x.kind == SV_OP_MEASURE_RESET;
            if (is_meas && terminal && j + 1 == xo.size()) continue;
            const int w = __builtin_popcount(qmask_of(x) | kRunMask);
            if (w > b->tile_q)
                return fail(SV_EUNSUPPORTED, "op %zu: its qubits and qubits 0..%d span %d qubits, "
                            "more than the %d-qubit tile", j, kCoalesceQ - 1, w, b->tile_q);
        }
    }

    // device program
    Plan plan;
    const uint32_t swz = b->dtype == SV_C128 ? 63u : 62u;
    const bool plain = b->mode == SV_MODE_PLAIN;
    if (plain)
        for (const XOp &x : xo)
            if (x.cond_mask != 0 || x.kind == SV_OP_BFUNC)
                return fail(SV_EUNSUPPORTED, "plain mode runs unconditional circuits only");
    if (plain) {  // list order, one pass and one group holding everything
        PassInfo pi;
        std::memset(&pi, 0, sizeof pi);
        pi.end_op = (uint32_t)xo.size();
        GroupInfo gi;
        std::memset(&gi, 0, sizeof gi);
        gi.end_op = (uint32_t)xo.size();
        gi.fallback = 1;
        for (uint32_t j = 0; j < xo.size(); ++j) {
            plan.order.push_back(j);
            plan.op_pass.push_back(0);
            plan.op_group.push_back(0);
        }
        plan.passes.push_back(pi);
        plan.groups.push_back(gi);
    } else {
        // a resident state is stored unswizzled. The plan depends only on the
        // ops' kinds, qubits, conditions and rule shapes and on the launch
        // shape, so a run that repeats them (waves of one job, serving
        // chunks) reuses a cached plan
        const uint32_t pswz = b->resident ? 0u : swz;
        const int span = b->dtype == SV_C128 ? 4 : 5;
        std::vector<int32_t> sig = {n, b->tile_q, b->reg_bits, b->resident, b->use_groups,
                                    (int32_t)pswz, span, terminal ? 1 : 0, (int32_t)xo.size()};
        sig.reserve(sig.size() + xo.size() * 8);
        for (const XOp &x : xo) {
            sig.push_back(x.kind);
            sig.push_back(x.rule >= 0 ? (rules[x.rule].kraus ? 2 : 1) * 64 + rules[x.rule].nq : -1);
            sig.push_back(x.cond_mask != 0 ? 1 : 0);
            sig.push_back((int32_t)x.q.size());
            for (int q : x.q) sig.push_back(q);
        }
        if (!plan_lookup(sig, plan)) {
            plan_program(n, b->tile_q, b->reg_bits, b->resident != 0, b->use_groups != 0, pswz, span, xo,
                         rules, terminal, plan);
            plan_store(std::move(sig), plan);
        }
    }
    const std::vector<PassInfo> &passes = plan.passes;
    std::vector<double> pool;
    std::vector<DevRule> drules(rules.size());
    for (size_t r = 0; r < rules.size(); ++r) rule_dev(rules[r], pool, drules[r]);
    std::vector<DevOp> dops(xo.size());
    for (size_t pos = 0; pos < plan.order.size(); ++pos) {
        const uint32_t j = plan.order[pos];
        const XOp &x = xo[j];
        DevOp &d = dops[pos];
        std::memset(&d, 0, sizeof d);
        d.r = j;
        d.pass = plan.op_pass[pos];
        d.group = plan.op_group[pos];
        d.nq = (uint8_t)x.q.size();
        const PassInfo &pi = passes[d.pass];
        const GroupInfo &gi = plan.groups[d.group];
        for (size_t t = 0; t < x.q.size() && t < 8; ++t) {
            d.q[t] = (uint8_t)x.q[t];
            int lb = 0;
            for (int a = 0; a < b->tile_q && a < 16; ++a)
                if (pi.tq[a] == x.q[t]) lb = a;
            d.lb[t] = (uint8_t)(b->resident ? x.q[t] : lb);
            int rb = 0;
            for (int a = 0; a < b->reg_bits && a < 8; ++a)
                if (gi.gpos[a] == d.lb[t]) rb = a;
            d.rb[t] = (uint8_t)rb;
        }
        d.cond_mask = x.cond_mask;
        d.cond_value = x.cond_value;
        if (x.cond_mask != 0 && x.kind != SV_OP_BFUNC) d.flags |= DF_COND;
        if (x.kind == SV_OP_BFUNC) {
            d.kind = DK_BFUNC;
            d.c[0] = (uint8_t)x.c[0];
        } else if (x.kind == -1 || x.kind == -2) {
            d.kind = x.kind == -1 ? DK_PAULI : DK_KRAUS;
            d.rule = (uint32_t)x.rule;
        } else if (x.kind == SV_OP_CX) {
            d.kind = DK_CX;
        } else if (x.kind == SV_OP_CZ) {
            d.kind = DK_CZ;
        } else if (x.kind == SV_OP_SWAP) {
            d.kind = DK_SWAP;
        } else if (x.kind == SV_OP_MEASURE || x.kind == SV_OP_RESET || x.kind == SV_OP_MEASURE_RESET) {
            d.kind = DK_MEASURE;
            if (x.kind != SV_OP_RESET) d.flags |= DF_RECORD;
            if (x.kind != SV_OP_MEASURE) d.flags |= DF_RESET;
            if (terminal && j + 1 == xo.size()) {
                d.flags |= DF_TERMINAL;
                d.nq = (uint8_t)n;
            }
            for (size_t t = 0; t < x.c.size() && t < 32; ++t) d.c[t] = (uint8_t)x.c[t];
        } else if (sweep && x.u3_index >= 0) {
            d.kind = DK_MAT1;
            d.flags |= DF_PARAM;       // matrices of every set follow the base pool
            d.mat = (uint32_t)(x.u3_index * 8);  // rebased below
        } else {
            d.kind = x.q.size() == 1 ? DK_MAT1 : DK_MATK;
            d.mat = (uint32_t)pool.size();
            bool diag = x.q.size() == 1 && x.mat[1] == 0.0 && x.mat[2] == 0.0;
            if (diag) d.flags |= DF_DIAG;
            for (const cd &v : x.mat) {
                pool.push_back(v.real());
                pool.push_back(v.imag());
            }
        }
    }
    uint32_t set_stride = 0;
    if (sweep) {
        int n_u3 = 0;
        for (const XOp &x : xo) n_u3 = std::max(n_u3, x.u3_index + 1);
        set_stride = (uint32_t)(n_u3 * 8);
        const uint64_t block = pool.size();
        if (block + (uint64_t)set_stride * n_sets > 0xffffffffull) return fail(SV_EINVAL, "sweep too large");
        for (size_t st = 0; st < n_sets; ++st)
            for (int u = 0; u < n_u3; ++u) {
                const double *a = params + (st * (size_t)n_u3 + u) * 3;
                for (const cd &v : gate_1q(SV_OP_U3, a)) {
                    pool.push_back(v.real());
                    pool.push_back(v.imag());
                }
            }
        for (DevOp &d : dops)
            if (d.flags & DF_PARAM) d.mat += (uint32_t)block;
    }
    if (pool.empty()) pool.push_back(0);
    // upload program
    const uint64_t ops_bytes = align_up(dops.size() * sizeof(DevOp), 256);
    const uint64_t pass_bytes = align_up(passes.size() * sizeof(PassInfo), 256);
    const uint64_t rule_bytes = align_up(std::max<size_t>(drules.size(), 1) * sizeof(DevRule), 256);
    const uint64_t pool_bytes = align_up(pool.size() * sizeof(double), 256);
    const uint64_t grp_bytes = align_up(plan.groups.size() * sizeof(GroupInfo), 256);
    const uint64_t prog_total = ops_bytes + pass_bytes + rule_bytes + pool_bytes + grp_bytes;
    if (prog_total > (uint64_t)b->program_bytes)
        return fail(SV_ENOMEM, "program needs %llu bytes; raise option program_bytes",
                    (unsigned long long)prog_total);
    std::vector<char> blob(prog_total, 0);
    std::memcpy(blob.data(), dops.data(), dops.size() * sizeof(DevOp));
    std::memcpy(blob.data() + ops_bytes, passes.data(), passes.size() * sizeof(PassInfo));
    if (!drules.empty()) std::memcpy(blob.data() + ops_bytes + pass_bytes, drules.data(), drules.size() * sizeof(DevRule));
    std::memcpy(blob.data() + ops_bytes + pass_bytes + rule_bytes, pool.data(), pool.size() * sizeof(double));
    std::memcpy(blob.data() + ops_bytes + pass_bytes + rule_bytes + pool_bytes, plan.groups.data(),
                plan.groups.size() * sizeof(GroupInfo));
    char *A = b->arena;
    const auto &L = b->lay;
    const bool use_graph = b->opt_graph != 0 && !b->noalloc_run && b->mode != SV_MODE_PLAIN;
    bool uploaded = true;
    if (use_graph) {
        const uint64_t h = blob_hash(blob);
        uploaded = !(h == b->prog_hash && b->prog_arena == A);
        b->prog_hash = h;
        b->prog_arena = A;
    } else {
        b->prog_hash = 0;  // the next graph run uploads again
    }
    if (uploaded)
        HIPCHK(hipMemcpyAsync(A + L.prog, blob.data(), blob.size(), hipMemcpyHostToDevice, b->stream));

    ExecParams P;
    std::memset(&P, 0, sizeof P);
    P.ops = (const DevOp *)(A + L.prog);
    P.passes = (const PassInfo *)(A + L.prog + ops_bytes);
    P.rules = (const DevRule *)(A + L.prog + ops_bytes + pass_bytes);
    P.pool = (const double *)(A + L.prog + ops_bytes + pass_bytes + rule_bytes);
    P.groups = (const GroupInfo *)(A + L.prog + ops_bytes + pass_bytes + rule_bytes + pool_bytes);
    P.slots = A + L.slots;
    P.slot_amps = 1ull << n;
    P.tile_sums = (double *)(A + L.tile_sums);
    P.shot_perm = (int32_t *)(A + L.perm);
    P.shot_tmp = (int32_t *)(A + L.tmp);
    P.memory = (uint64_t *)(A + L.memory);
    P.margins = (uint64_t *)(A + L.margins);
    P.queue = (BranchRec *)(A + L.queue);
    P.ready = (uint32_t *)(A + L.ready);
    P.ctl = (Control *)(A + L.ctl);
    P.free_slots = (int32_t *)(A + L.free_slots);
    P.waiting = (int32_t *)(A + L.waiting);
    P.dump = b->dump_shot >= 0 ? (void *)(A + L.dump) : nullptr;
    P.seed = seed;
    P.shot_base = (uint64_t)b->shot_offset;
    P.n_shots = b->shots;
    P.dump_shot = b->dump_shot;
    P.spin_limit = (unsigned long long)b->spin_ms * (unsigned long long)b->wallclock_khz;
    P.spin_elapsed = (int32_t)b->spin_elapsed;
    P.ro01 = ro01;
    P.ro10 = ro10;
    P.n_ops = (int32_t)dops.size();
    P.n_qubits = n;
    P.tile_q = b->tile_q;
    P.n_slots = b->slots;
    P.queue_cap = (int32_t)b->shots;
    P.branch_mode = b->mode == SV_MODE_BRANCH;
    P.private_slots = (!b->resident && b->mode == SV_MODE_BATCH) ? 1 : 0;
    P.resident = b->resident;
    P.use_groups = b->use_groups;
    P.swz = swz;
    P.nbuf = b->nbuf;
    P.stage_cap = b->stage_cap;
    P.n_rules = (int32_t)drules.size();
    {
        int terms = 0;
        for (const DevRule &r : drules)
            if (!r.is_kraus) terms += (int)r.n_terms;
        P.stage_rules = (b->stage_cap > 0 && drules.size() <= (size_t)kStageRules &&
                         terms <= kStageTerms) ? 1 : 0;
    }
    P.set_stride = set_stride;
    P.shots_per_set = sweep ? (uint32_t)((uint64_t)b->shots / n_sets) : 1u;
    {
        // complex64 one-qubit micro-ops on the matrix cores unless the vector
        // ALU is asked for: measured faster on the 20-qubit workload (2.6
        // one-qubit gates per register group; 732 against 772 ms per 1024
        // shots) and on the 26-qubit one (5.6 per group)
        const int mf = (b->dtype == SV_C64 && b->use_groups && b->opt_mfma != 1) ? 1 : 0;
        P.mfma1 = mf;
        b->mfma = mf;
    }

    if (plain) {
        double *scratch = (double *)(A + L.tile_sums);
        double *chunk = scratch + (size_t)kPlainRedBlocks * 17;
        void *cell = chunk + (((1ull << n) + 255) / 256);
        HIPCHK(ev_record(b->ev0, b->stream));
        HIPCHK(ev_record(b->ev2, b->stream));
        HIPCHK(svb_plain_run(b->dtype == SV_C128, P.ops, dops.data(), P.n_ops, P.rules, drules.data(),
                             P.pool, n, (uint64_t)b->shots, P.shot_base, seed, P.slots, P.memory,
                             P.margins, scratch, kPlainRedBlocks, chunk, cell, ro01, ro10,
                             b->stream));
        HIPCHK(ev_record(b->ev3, b->stream));
        HIPCHK(ev_record(b->ev1, b->stream));
        HIPCHK(ev_wait(b->ev1, b->stream));
        float ms = 0, ems = 0;
        HIPCHK(ev_ms(&ms, b->ev0, b->ev1));
        HIPCHK(ev_ms(&ems, b->ev2, b->ev3));
        sv_stats &st = b->stats;
        std::memset(&st, 0, sizeof st);
        st.kernel_ms = ms;
        st.exec_ms = ems;
        st.exec_launches = 1;
        st.expanded_ops = xo.size();
        st.gate_count = gate_count;
        st.workers = 1;
        st.slots = 1;
        st.tile_qubits = (uint32_t)n;
        // state sweeps per shot: a gate reads and writes the state; a Kraus
        // channel or a measurement adds a read-only reduction sweep; a Pauli
        // channel moves data only when it draws a non-identity string
        // (rare, not counted: the byte figure is a lower bound)
        uint64_t rw = 0, ro = 0;
        for (const XOp &x : xo) {
            if (x.kind == -1 || x.kind == SV_OP_BFUNC) continue;
            ++rw;
            if (x.kind == -2 || x.kind == SV_OP_MEASURE || x.kind == SV_OP_RESET ||
                x.kind == SV_OP_MEASURE_RESET)
                ++ro;
        }
        st.passes = (uint64_t)b->shots * (rw + ro);
        st.amp_bytes = (uint64_t)b->shots * (2 * rw + ro) * state_bytes(b);
        b->have_results = true;
        b->have_stats = true;
        b->have_dump = false;
        return SV_OK;
    }

    const bool branch = P.branch_mode != 0;
    const int root_slot = (branch && !b->resident) ? 0 : -1;
    const int n_free = branch ? (b->resident ? b->slots : b->slots - 1) : 0;
    uint64_t acc[ST_COUNT] = {0};
    uint64_t restarts = 0;
    HIPCHK(ev_record(b->ev0, b->stream));
    if (!use_graph) HIPCHK(svb_launch_init(&P, 0, (int)b->shots, root_slot, n_free, b->stream));
    double exec_ms = 0;
    uint32_t exec_launches = 0;
    for (;;) {
        HIPCHK(ev_record(b->ev2, b->stream));
        if (use_graph && exec_launches == 0) {
            // initialisation + executor from the graph (exec_ms then includes
            // the initialisation kernel, a few microseconds)
            s = graph_run(b, P, root_slot, n_free);
            if (s != SV_OK) return s;
        } else {
            HIPCHK(svb_launch_exec(&P, b->dtype == SV_C128, b->reg_bits, b->workers, b->stream));
        }
        HIPCHK(ev_record(b->ev3, b->stream));
        Control ctl;
        HIPCHK(hipMemcpyAsync(&ctl, P.ctl, sizeof ctl, hipMemcpyDeviceToHost, b->stream));
        HIPCHK(hipStreamSynchronize(b->stream));
        float lms = 0;
        HIPCHK(ev_ms(&lms, b->ev2, b->ev3));
        exec_ms += lms;
        ++exec_launches;
        if (ctl.error) return fail(SV_EDEVICE, "device executor failed (flags 0x%x)", ctl.error);
        for (int i = 0; i < ST_COUNT; ++i) acc[i] += ctl.stat[i];
        if (ctl.wait_count == 0) break;
        ++restarts;
        HIPCHK(svb_launch_restart(&P, (int)ctl.wait_count, b->stream));
        HIPCHK(svb_launch_init(&P, 1, (int)ctl.wait_count, root_slot, n_free, b->stream));
    }
    HIPCHK(ev_record(b->ev1, b->stream));
    HIPCHK(ev_wait(b->ev1, b->stream));
    float ms = 0;
    HIPCHK(ev_ms(&ms, b->ev0, b->ev1));

    sv_stats &st = b->stats;
    std::memset(&st, 0, sizeof st);
    st.kernel_ms = ms;
    st.passes = acc[ST_PASSES];
    st.amp_bytes = acc[ST_BYTES];
    st.reductions = acc[ST_REDUCTIONS];
    st.branches = acc[ST_BRANCHES];
    st.restarts = restarts;
    st.waiting_shots = acc[ST_WAITING];
    st.expanded_ops = xo.size();
    st.gate_count = gate_count;
    st.workers = (uint32_t)b->workers;
    st.slots = (uint32_t)b->slots;
    st.tile_qubits = (uint32_t)b->tile_q;
    st.tile_buffers = (uint32_t)b->nbuf;
    st.static_passes = (uint32_t)passes.size();
    st.flops = acc[ST_FLOPS];
    st.exec_ms = exec_ms;
    st.groups = acc[ST_GROUPS];
    st.uops = acc[ST_UOPS];
    st.near_ties = acc[ST_NEARTIES];
    st.exec_launches = exec_launches;
    st.graph_replays = use_graph ? 1u : 0u;
    st.program_uploads = uploaded ? 1u : 0u;
    st.mfma = (uint32_t)b->mfma;
    b->have_results = true;
    b->have_stats = true;
    b->have_dump = b->dump_shot >= 0;
    return SV_OK;
}

sv_status sv_run_circuit(sv_batch *b, const sv_op *ops, size_t n_ops, const sv_noise_model *nm,
                         uint64_t seed)
{
    return run_impl(b, ops, n_ops, nm, seed, nullptr, 1);
}

sv_status sv_run_sweep(sv_batch *b, const sv_op *ops, size_t n_ops, const sv_noise_model *nm,
                       uint64_t seed, const double *params, size_t n_sets)
{
    if (!params) return fail(SV_EINVAL, "params is NULL");
    return run_impl(b, ops, n_ops, nm, seed, params, n_sets);
}

// Fit the state slots (and in batch mode the workgroups that own them, one
// slot each) into an arena of cap bytes; the rest of the layout is fixed by
// the shot count and the options.
static sv_status fit_arena(sv_batch *b, uint64_t cap)
{
    layout(b);
    while (b->lay.total > cap && b->slots > 1) {
        const uint64_t over = b->lay.total - cap;
        const int64_t drop = std::max<int64_t>(1, (int64_t)((over + state_bytes(b) - 1) / state_bytes(b)));
        b->slots = (int)std::max<int64_t>(1, (int64_t)b->slots - drop);
        if (b->mode == SV_MODE_BATCH && !b->resident) b->workers = b->slots;
        layout(b);
    }
    if (b->lay.total > cap)
        return fail(SV_ENOMEM, "needs %llu device bytes with one state slot, more than the "
                    "%llu of the no-allocation buffer (fewer shots or a smaller program_bytes "
                    "may fit)", (unsigned long long)b->lay.total, (unsigned long long)cap);
    return SV_OK;
}

sv_status sv_run_circuit_noalloc(sv_batch *b, const sv_op *ops, size_t n_ops,
                                 const sv_noise_model *nm, uint64_t seed, void *hip_stream,
                                 uint64_t *memory_out, size_t n_memory)
{
    if (!b || !memory_out) return fail(SV_EINVAL, "NULL argument");
    if (b->attached) return fail(SV_ESTATE, "the handle has an attached arena: use sv_run_circuit");
    if (n_memory != (size_t)b->shots)
        return fail(SV_EINVAL, "n_memory=%zu, shots=%lld", n_memory, (long long)b->shots);
    void *ptr = nullptr;
    uint64_t cap = 0;
    HIPCHK(svb_noalloc_scratch(&ptr, &cap));
    b->no_counts = true;
    sv_status s = derive(b);
    if (s == SV_OK) s = fit_arena(b, cap);
    if (s == SV_OK) {
        b->arena = (char *)ptr;
        b->arena_bytes = cap;
        b->stream = (hipStream_t)hip_stream;
        b->attached = true;
        b->noalloc_run = true;
        s = run_impl(b, ops, n_ops, nm, seed, nullptr, 1);
        b->noalloc_run = false;
        if (s == SV_OK) {
            const hipError_t e1 = hipMemcpyAsync(memory_out, b->arena + b->lay.memory, n_memory * 8,
                                                 hipMemcpyDeviceToHost, b->stream);
            const hipError_t e2 = e1 == hipSuccess ? hipStreamSynchronize(b->stream) : e1;
            if (e2 != hipSuccess)
                s = fail(SV_EDEVICE, "copy of the registers: %s", hipGetErrorString(e2));
        }
    }
    // every no-allocation call on this device shares the buffer: nothing of
    // this run stays readable through the handle but its statistics
    b->attached = false;
    b->arena = nullptr;
    b->arena_bytes = 0;
    b->stream = nullptr;
    b->no_counts = false;
    b->have_results = false;
    b->have_dump = false;
    if (s != SV_OK) b->have_stats = false;
    return s;
}

sv_status sv_sample_counts(sv_batch *b, uint64_t *keys, uint64_t *counts, size_t capacity,
                           size_t *n_unique)
{
    if (!b || !n_unique) return fail(SV_EINVAL, "NULL argument");
    if (!b->have_results) return fail(SV_ESTATE, "no results: run a circuit first");
    char *A = b->arena;
    const auto &L = b->lay;
    HIPCHK(svb_counts((const uint64_t *)(A + L.memory), b->shots, A + L.counts_tmp,
                      svb_counts_temp_bytes(b->shots), (uint64_t *)(A + L.keys_sorted),
                      (uint64_t *)(A + L.uniq), (uint32_t *)(A + L.cnt), (uint32_t *)(A + L.nuniq),
                      b->stream));
    uint32_t nu = 0;
    HIPCHK(hipMemcpyAsync(&nu, A + L.nuniq, 4, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    *n_unique = nu;
    if (nu > capacity) return fail(SV_EINVAL, "capacity %zu < %u distinct keys", capacity, nu);
    if (nu) {
        if (!keys || !counts) return fail(SV_EINVAL, "NULL output arrays");
        std::vector<uint32_t> c32(nu);
        HIPCHK(hipMemcpyAsync(keys, A + L.uniq, (size_t)nu * 8, hipMemcpyDeviceToHost, b->stream));
        HIPCHK(hipMemcpyAsync(c32.data(), A + L.cnt, (size_t)nu * 4, hipMemcpyDeviceToHost, b->stream));
        HIPCHK(hipStreamSynchronize(b->stream));
        for (uint32_t i = 0; i < nu; ++i) counts[i] = c32[i];
    }
    return SV_OK;
}

sv_status sv_get_memory(sv_batch *b, uint64_t *out, size_t n)
{
    if (!b || !out) return fail(SV_EINVAL, "NULL argument");
    if (!b->have_results) return fail(SV_ESTATE, "no results: run a circuit first");
    if (n != (size_t)b->shots) return fail(SV_EINVAL, "n=%zu, shots=%lld", n, (long long)b->shots);
    HIPCHK(hipMemcpyAsync(out, b->arena + b->lay.memory, n * 8, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    return SV_OK;
}

sv_status sv_get_margins(sv_batch *b, double *out, size_t n)
{
    if (!b || !out) return fail(SV_EINVAL, "NULL argument");
    if (!b->have_results) return fail(SV_ESTATE, "no results: run a circuit first");
    if (n != (size_t)b->shots) return fail(SV_EINVAL, "n=%zu, shots=%lld", n, (long long)b->shots);
    HIPCHK(hipMemcpyAsync(out, b->arena + b->lay.margins, n * 8, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    return SV_OK;
}

sv_status sv_get_state(sv_batch *b, double *amps, size_t n_amps)
{
    if (!b || !amps) return fail(SV_EINVAL, "NULL argument");
    if (!b->have_dump) return fail(SV_ESTATE, "no state kept: set option dump_shot and run");
    if (n_amps != (1ull << b->n)) return fail(SV_EINVAL, "n_amps=%zu, expected %llu", n_amps, 1ull << b->n);
    HIPCHK(hipMemcpyAsync(amps, b->arena + b->lay.dump, n_amps * 16, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    return SV_OK;
}

sv_status sv_get_stats(sv_batch *b, sv_stats *out)
{
    if (!b || !out) return fail(SV_EINVAL, "NULL argument");
    if (!b->have_stats) return fail(SV_ESTATE, "no results: run a circuit first");
    *out = b->stats;
    return SV_OK;
}

// Host-only introspection of the execution plan (tests): device order of the
// expanded ops (as expanded-list indices), their pass and group, each pass's
// tile-qubit mask and each group's register-qubit count (-1: LDS group).
sv_status svb_debug_plan(int n_qubits, int tile_q, int reg_bits, const sv_op *ops, size_t n_ops,
                         const sv_noise_model *nm, int32_t *order, int32_t *op_pass,
                         int32_t *op_group, uint32_t *pass_mask, int32_t *group_width,
                         size_t cap, size_t *n_out, size_t *n_passes, size_t *n_groups)
{
    sv_batch tmp;
    tmp.n = n_qubits;
    tmp.shots = 1;
    std::vector<Rule> rules;
    std::vector<XOp> xo;
    double ro01, ro10;
    uint64_t gc;
    sv_status s = validate_and_expand(&tmp, ops, n_ops, nm, rules, xo, ro01, ro10, gc);
    if (s != SV_OK) return s;
    bool terminal = false;
    if (!xo.empty()) {
        const XOp &last = xo.back();
        if (last.kind == SV_OP_MEASURE && (int)last.q.size() == n_qubits) {
            terminal = true;
            for (int t = 0; t < n_qubits; ++t) terminal = terminal && last.q[t] == t;
            terminal = terminal && last.cond_mask == 0;
        }
    }
    const bool resident = n_qubits <= tile_q;
    Plan plan;
    plan_program(n_qubits, resident ? n_qubits : tile_q, reg_bits, resident, reg_bits > 0,
                 resident ? 0u : 62u, 5, xo, rules, terminal, plan);
    *n_out = plan.order.size();
    *n_passes = plan.passes.size();
    *n_groups = plan.groups.size();
    if (plan.order.size() > cap || plan.passes.size() > cap || plan.groups.size() > cap)
        return fail(SV_EINVAL, "capacity %zu too small", cap);
    for (size_t i = 0; i < plan.order.size(); ++i) {
        order[i] = (int32_t)plan.order[i];
        op_pass[i] = (int32_t)plan.op_pass[i];
        op_group[i] = (int32_t)plan.op_group[i];
    }
    for (size_t p = 0; p < plan.passes.size(); ++p) pass_mask[p] = plan.passes[p].tmask;
    for (size_t g = 0; g < plan.groups.size(); ++g) {
        if (plan.groups[g].fallback) {
            group_width[g] = -1;
        } else {
            uint32_t m = 0;
            for (uint32_t j = plan.groups[g].first_op; j < plan.groups[g].end_op; ++j)
                m |= qmask_of(xo[plan.order[j]]);
            group_width[g] = __builtin_popcount(m);
        }
    }
    return SV_OK;
}

sv_status sv_batch_destroy(sv_batch *b)
{
    if (!b) return SV_OK;
    if (b->ev0) (void)hipEventDestroy(b->ev0);
    if (b->ev1) (void)hipEventDestroy(b->ev1);
    if (b->ev2) (void)hipEventDestroy(b->ev2);
    if (b->ev3) (void)hipEventDestroy(b->ev3);
    graph_drop(b);
    delete b;
    return SV_OK;
}

}  // extern "C"
