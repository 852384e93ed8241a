// Device program of one circuit: op records, static pass plan, parameter
// pool, and the control/queue records of the persistent executor. Shared by
// the host runtime (runtime.cpp) and the kernels (kernels.hip).
#pragma once
#include <stdint.h>

namespace svb {

constexpr int kWG = 256;             // threads per executor workgroup
constexpr int kWGBits = 8;           // log2(kWG)
static_assert((1 << kWGBits) == kWG, "kWGBits is log2(kWG)");
constexpr int kMaxPassOps = 512;     // ops applied in one tile sweep
constexpr int kMaxPassGroups = 64;   // register groups in one sweep
constexpr int kMaxPassUops = 384;    // register micro-ops in one sweep
constexpr int kPassMatBytes = 6144;  // LDS bytes for the fused 2x2 matrices of one sweep
constexpr int kMaxKraus = 16;        // matrices per Kraus channel
constexpr int kMaxDenseQ = 5;        // qubits of a dense matrix (unitary, Kraus channel)
constexpr int kMaxPauliQ = 5;        // qubits of a Pauli channel
constexpr int kMaxPauliTerms = 1024; // terms of a Pauli channel (4^5)
constexpr int kMaxMeasQ = 4;         // qubits of a non-terminal measure
constexpr int kMaxRed = 1 + 16;      // norm + up to 16 outcome sums
constexpr int kCoalesceQ = 4;        // low qubits always inside a tile
constexpr double kNearTie = 1e-9;    // relative decision margin counted as a near-tie
constexpr uint64_t kInfBits = 0x7FF0000000000000ull;  // +inf as double bits
constexpr uint32_t kRunMask = (1u << kCoalesceQ) - 1;  // contiguous run of a tile in HBM
constexpr int kMaxTileQ = 14;
constexpr int kStageOps = 128;       // ops of a pass staged in LDS (resident states)
constexpr int kStageRules = 16;      // noise rules staged in LDS with them
constexpr int kStageTerms = 256;     // Pauli terms (thresholds and codes) staged in LDS

// Device op kinds (after noise-site expansion).
enum DevKind : uint16_t {
    DK_MAT1 = 1,     // 2x2 matrix on lb[0]
    DK_MATK = 2,     // dense 2^nq x 2^nq matrix (nq = 2..5) on lb[0..nq-1];
                     // bit t of its row/column index <-> lb[t]
    DK_CX = 3,       // control lb[0], target lb[1]
    DK_CZ = 4,
    DK_SWAP = 5,
    DK_PAULI = 6,    // Pauli channel of rule `rule`
    DK_KRAUS = 7,    // Kraus channel of rule `rule`
    DK_MEASURE = 8,  // measure / reset / measure+reset of q[0..nq-1]
    DK_BFUNC = 9,    // clbit c[0] <- ((creg & cond_mask) == cond_value)
};

// decision of an op whose condition fails (it is skipped)
constexpr int kSkip = -2;

enum DevFlags : uint8_t {
    DF_DIAG = 1,      // DK_MAT1: off-diagonal entries are zero
    DF_RECORD = 2,    // DK_MEASURE: write clbits
    DF_RESET = 4,     // DK_MEASURE: return measured 1s to |0>
    DF_TERMINAL = 8,  // DK_MEASURE: last op, all qubits in order (sampling)
    DF_COND = 16,     // runs only for shots with (creg & cond_mask) == cond_value
    DF_PARAM = 32,    // DK_MAT1 of a swept U3: matrix of set s at mat + s * set_stride
};

struct DevOp {
    uint16_t kind;
    uint8_t nq;
    uint8_t flags;
    uint32_t r;          // index in the expanded op list (Philox counter word)
    uint32_t pass;       // static pass holding this op
    uint32_t mat;        // pool offset (doubles) of this op's matrix
    uint32_t rule;       // noise rule index (DK_PAULI / DK_KRAUS)
    uint32_t group;      // register group holding this op
    uint8_t q[8];        // physical qubits
    uint8_t lb[8];       // tile-local bit of each qubit in its static pass
    uint8_t rb[8];       // register bit of each qubit in its group
    uint8_t c[32];       // clbits (terminal measure: clbit of qubit t)
    uint64_t cond_mask;  // DF_COND / DK_BFUNC: predicate on the classical register
    uint64_t cond_value;
};

// A register group: consecutive ops of a pass whose qubits lie on at most
// r = log2(amplitudes per thread) tile bits. Each thread gathers the 2^r
// amplitudes that differ in those bits from LDS into registers, applies the
// group's ops there and scatters them back.
struct GroupInfo {
    uint32_t first_op, end_op;  // ops [first_op, end_op)
    uint32_t fallback;          // 1: ops run as LDS sweeps (measure, 4x4 ops)
    uint32_t pad;
    uint8_t gpos[8];            // register bit j -> tile bit
    uint8_t cpos[16];           // thread-index bit i -> tile bit
};

// Per-rule channel data in the pool.
struct DevRule {
    uint32_t is_kraus;
    uint32_t nq;
    uint32_t n_terms;
    uint32_t thr;        // Pauli: pool offset of cumulative thresholds (doubles)
    uint32_t mats;       // Kraus: pool offset of matrices (fp64 complex)
    uint32_t diag_mm;    // Kraus: every K^dagger K is diagonal
    double lam_min0;     // Kraus: smallest eigenvalue of K0^dagger K0
    uint32_t codes;      // Pauli: pool offset of the term codes, one double per term
                         // holding x | z << 8 | ny << 16 (bit t of x: X or Y on gate
                         // qubit t; of z: Z or Y; ny: number of Y; 0: identity)
    uint32_t scalar_mask;// Kraus: bit j set if matrix j is a multiple of the identity
};

struct PassInfo {
    uint32_t first_op, end_op;  // ops [first_op, end_op)
    uint32_t tmask;             // physical qubits inside the tile
    uint32_t contiguous;        // tile qubits are 0..k-1
    uint8_t tq[16];             // tile qubits, ascending (k entries)
    uint8_t gq[32];             // remaining qubits, ascending (n-k entries)
};

// Work-queue record: a state (slot) shared by shots shot_perm[lo..hi).
struct BranchRec {
    int32_t slot;       // state slot, -1: none (fresh |0> in LDS)
    int32_t lo, hi;     // shot range in shot_perm
    int32_t cursor;     // next op to apply
    int32_t pending;    // decided outcome of op[cursor], -1: none
    int32_t flags;      // bit0: slot content is the fresh |0> state (not written)
    double scale;       // renormalisation applied with the pending op
    double norm_lb;     // lower bound of the state's squared norm
};

enum CtlStat {
    ST_PASSES = 0, ST_BYTES, ST_REDUCTIONS, ST_BRANCHES, ST_WAITING,
    ST_FLOPS, ST_SPLITS, ST_GROUPS, ST_UOPS, ST_NEARTIES, ST_COUNT
};

struct Control {
    uint32_t q_head;        // tickets handed out
    uint32_t q_tail;        // records reserved
    int32_t outstanding;    // records pushed and not finished
    uint32_t error;         // device failure flags (see kErr*)
    uint32_t lock;          // slot stack lock
    int32_t free_top;       // free slots on the stack
    uint32_t wait_count;    // shots on the waiting list
    uint32_t n_initial;     // records present at launch
    unsigned long long stat[ST_COUNT];
    uint32_t done_workers;
    uint32_t heartbeat;     // bumped by every workgroup at each sweep and record end
    uint32_t pad[6];
};

constexpr uint32_t kErrTimeout = 1;
constexpr uint32_t kErrQueue = 2;
constexpr uint32_t kErrLock = 4;
constexpr uint32_t kErrState = 8;
constexpr uint32_t kErrFuse = 16;   // plan-time fusion overran its counted room (internal)

struct ExecParams {
    const DevOp *ops;
    const PassInfo *passes;
    const DevRule *rules;
    const GroupInfo *groups;
    const double *pool;
    void *slots;             // n_slots states, slot_amps amplitudes apart
    uint64_t slot_amps;
    double *tile_sums;       // per worker 2^(n-k) doubles (terminal sampling)
    int32_t *shot_perm;
    int32_t *shot_tmp;
    uint64_t *memory;
    BranchRec *queue;
    uint32_t *ready;
    Control *ctl;
    int32_t *free_slots;
    int32_t *waiting;
    void *dump;              // normalised state of dump_shot (complex)
    uint64_t *margins;       // per shot: bits of its smallest relative decision margin
                             // (a non-negative double, +inf without a decision)
    uint64_t seed;
    uint64_t shot_base;      // global id of local shot 0 (Philox counter)
    int64_t n_shots;
    int64_t dump_shot;
    unsigned long long spin_limit;   // wall-clock ticks a work-queue wait may last
                                     // without any workgroup making progress
    int32_t spin_elapsed;    // 1: the bound counts from the start of the wait,
                             // whatever the other workgroups do
    double ro01, ro10;
    int32_t n_ops;
    int32_t n_qubits;
    int32_t tile_q;          // k (== n_qubits when the state lives in LDS)
    int32_t n_slots;
    int32_t queue_cap;
    int32_t branch_mode;     // 1: shots may split (work queue with pushes)
    int32_t private_slots;   // 1: worker w uses slot w (batch mode, n > k)
    int32_t resident;        // 1: whole state in LDS (n <= k)
    int32_t use_groups;      // 1: streamed passes run register groups
    uint32_t swz;            // LDS swizzle mask of streamed passes
    uint32_t set_stride;     // parameter sweep: pool doubles between sets (0: none)
    uint32_t shots_per_set;  // parameter sweep: shots of each set
    int32_t nbuf;            // LDS tile buffers of streamed grouped passes (1, or 2:
                             // the next tile is fetched while this one computes)
    int32_t stage_cap;       // > 0: a pass's op records (at most this many) and their
                             // one-qubit matrices are copied to LDS before it is planned
    int32_t n_rules;         // noise rules of the program
    int32_t stage_rules;     // 1: the rules and their Pauli tables are copied to LDS once
    int32_t mfma1;           // 1: fused non-diagonal one-qubit micro-ops of complex64
                             // register groups run on the matrix cores
};

}  // namespace svb
