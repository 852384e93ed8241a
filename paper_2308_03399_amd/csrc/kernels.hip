// Persistent multi-shot executor for gfx950.
//
// One workgroup owns one state at a time and runs the whole expanded op list
// on it (batch-shots of Sec. IV-A: all shots in one launch; shot-branching of
// Sec. IV-B: a state shared by a range of shots, split when their draws
// disagree). Ops are applied in LDS tiles of 2^k amplitudes: a tile holds
// the k "tile qubits" of the current pass (always including qubits 0..3 so
// that global accesses are 128-byte runs) and one fixed value of the other
// qubits. When the whole state fits in LDS (n <= k) it never leaves LDS.
//
// Random decisions are taken per shot from Philox4x32-10 draws keyed by
// (seed, shot, expanded-op index):
//  * Pauli channels: first table entry whose running sum exceeds u.
//  * Kraus channels: first K_j whose running sum of ||K_j psi||^2 exceeds
//    u*||psi||^2 (FP64 reduction over the state). When u is below the
//    smallest eigenvalue of K_0^dagger K_0 the choice is K_0 whatever the
//    state is, so no reduction is needed; K_0 is then applied without
//    renormalisation (every later decision compares against the norm of the
//    same reduction, so the scale cancels).
//  * Measure: FP64 outcome probabilities, first running sum above u*N.
//  * Final measurement of all qubits: chunked FP64 prefix sums (tile sums,
//    then an in-tile scan) and a search per shot (sampling technique).
// Reductions use a fixed tree: thread-sequential, wave butterfly, then the
// four waves in order, then tiles in order, so results do not depend on the
// batch or the launch shape.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "program.h"

namespace svb {

// Amplitudes and 16-byte chunks as clang vector types (usable through
// address-space-qualified pointers, unlike the HIP vector classes).
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <class R> struct V2;
template <> struct V2<float> { using T = f32x2; };
template <> struct V2<double> { using T = f64x2; };

// LDS (address space 3) and global (address space 1) pointers, so that tile
// accesses compile to ds_* and global_* instructions rather than flat ones.
template <class T> using lds = __attribute__((address_space(3))) T;
template <class T> using gbl = __attribute__((address_space(1))) T;
// read-only program data (groups, passes) seen through the constant
// address space: uniform reads become scalar loads, which leave the vector
// memory counter to the tile copies in flight
template <class T> using cst = __attribute__((address_space(4))) T;
// a pointer every lane holds the same value of, made uniform (scalar)
template <class T>
__device__ __forceinline__ gbl<T> *uni_ptr(gbl<T> *p)
{
    const uint64_t a = (uint64_t)p;
    const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    return (gbl<T> *)(lo | (hi << 32));
}

template <class T>
__device__ __forceinline__ const cst<T> *to_const(const T *p)
{
    const uint64_t a = (uint64_t)p;
    const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    return (const cst<T> *)(lo | (hi << 32));
}

// ------------------------------------------------------------------ RNG
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 multiplies with the published multipliers, the key bumped by
// the two Weyl constants between rounds.
__device__ __forceinline__ double philox_u01(uint64_t seed, uint64_t shot,
                                             uint32_t r, uint32_t d)
{
    uint32_t x0 = (uint32_t)shot, x1 = (uint32_t)(shot >> 32), x2 = r, x3 = d;
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        const uint32_t a = 0xD2511F53u * x0, ah = __umulhi(0xD2511F53u, x0);
        const uint32_t b = 0xCD9E8D57u * x2, bh = __umulhi(0xCD9E8D57u, x2);
        const uint32_t y0 = bh ^ x1 ^ k0, y2 = ah ^ x3 ^ k1;
        x0 = y0; x1 = b; x2 = y2; x3 = a;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    const uint64_t v = ((uint64_t)(x0 >> 5) << 26) | (uint64_t)(x1 >> 6);
    return (double)v * 0x1.0p-53;
}

// ------------------------------------------------------------------ misc
__device__ __forceinline__ uint32_t ins0(uint32_t p, uint32_t b)
{
    const uint32_t lo = p & ((1u << b) - 1u);
    return ((p ^ lo) << 1) | lo;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Workgroup barrier that orders LDS accesses only. __syncthreads() also
// waits for the wave's global memory operations, which would stall on the
// asynchronous tile copy in flight.
__device__ __forceinline__ void lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// wait until every vector memory operation of this wave has completed
// (the asynchronous global->LDS copies included)
__device__ __forceinline__ void wait_vm() { __builtin_amdgcn_s_waitcnt(0x0F70); }

__device__ __forceinline__ uint32_t ld_rlx(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t ld_rlx_i(const int32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rel(uint32_t *p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

template <class R> struct Mat2 { R r[4], i[4]; };

// Pauli term code of a drawn term: x | z << 8 | ny << 16 (0: identity).
__device__ __forceinline__ uint32_t pauli_code(const ExecParams &P, const DevRule &ru, int d)
{
    return (uint32_t)P.pool[ru.codes + (uint32_t)d];
}

template <class R>
__device__ __forceinline__ Mat2<R> load_m2(const double *m, double s)
{
    Mat2<R> o;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        o.r[e] = (R)(m[2 * e] * s);
        o.i[e] = (R)(m[2 * e + 1] * s);
    }
    return o;
}

// acc + (mr + i mi) * v
template <class A, class R>
__device__ __forceinline__ A cmac(A acc, R mr, R mi, A v)
{
    acc.x = fma(mr, v.x, fma(-mi, v.y, acc.x));
    acc.y = fma(mr, v.y, fma(mi, v.x, acc.y));
    return acc;
}

template <class A, class R>
__device__ __forceinline__ A cmul(R mr, R mi, A v)
{
    A o;
    o.x = fma(mr, v.x, -mi * v.y);
    o.y = fma(mr, v.y, mi * v.x);
    return o;
}

// Exact multiplication by (-i)^ny.
template <class A>
__device__ __forceinline__ A phase_ny(A v, uint32_t ny)
{
    A o;
    switch (ny & 3u) {
    case 0: o = v; break;
    case 1: o.x = v.y; o.y = -v.x; break;
    case 2: o.x = -v.x; o.y = -v.y; break;
    default: o.x = -v.y; o.y = v.x; break;
    }
    return o;
}

template <class A>
__device__ __forceinline__ A neg_if(A v, uint32_t odd)
{
    if (odd & 1u) { v.x = -v.x; v.y = -v.y; }
    return v;
}

template <class A>
__device__ __forceinline__ double abs2d(A v)
{
    const double x = (double)v.x, y = (double)v.y;
    return fma(x, x, y * y);
}

// ------------------------------------------------------------------ shared
enum StopKind { STOP_NONE = 0, STOP_REDUCE = 1, STOP_SPLIT = 2,
                STOP_TERMINAL = 3, STOP_END = 4 };
enum Status { ST_WORK = 0, ST_EXIT = 1 };

struct WgShared {
    BranchRec rec;
    int status;
    int slot;        // state slot (streamed mode), -1 if none
    int fresh;       // slot holds the virtual |0..0> state
    int lo, hi;      // shot range
    int cursor;
    int pending;
    double first_scale;
    double norm_lb;
    int start, end, stop, stop_op;
    int omin, omax, anyhigh;
    int n_groups;
    int grp_o[16];
    int grp_lo[16];
    int grp_hi[16];
    int tot[16];
    int alloc_slot;
    int wait_base;
    int dump_here;
    double red[kMaxRed];
    double wred[kMaxRed][kWG / 64];
    double tsum_n;
    int term_tile;
    int split_cond;  // STOP_SPLIT: the stopping op's condition differs between shots
    int n_distinct;  // terms drawn in a record split by term rank
    int n_ug;
    uint64_t pass_flops;
    unsigned long long st[ST_COUNT];
};

// Register micro-op built at plan time (fused 2x2 matrices, permutations).
// UK_MAT1R: a 2x2 matrix whose top-left entry is real (a U3 gate, alone or
// with diagonal noise factors), two multiplications fewer per pair.
// UK_MAT1M: a 2x2 matrix applied on the matrix cores (complex64)
enum UKind : uint8_t { UK_MAT1 = 1, UK_DIAG1 = 2, UK_CX = 3, UK_CZ = 4, UK_SWAP = 5, UK_MAT1R = 6,
                       UK_MAT1M = 7 };
// Dispatch code of a micro-op, one dense number per (kind, register bits)
// so that the register-group loop branches once: one-qubit kinds on bit J
// at kCodeMat1/kCodeMat1R/kCodeDiag1 + J, two-qubit kinds on (c, t) at
// kCodeCX/kCodeCZ/kCodeSwap + 6c + t, matrix-core one-qubit kinds at
// kCodeMat1M + J, and kCodeCopy (no change).
constexpr uint32_t kCodeMat1 = 0, kCodeMat1R = 8, kCodeDiag1 = 16, kCodeCX = 24, kCodeCZ = 60,
                   kCodeSwap = 96, kCodeMat1M = 132, kCodeCopy = 255;
struct UOp {
    uint8_t kind, j0, j1, code;
    uint16_t mat, pad2;
};
// A register group of the pass. flags bit 0: an LDS group (fallback);
// bit 26: the group ends with a permutation of its register bits that is
// applied by where the results are stored, not by moving them: bits
// 1 + 5a .. 5 + 5a hold the image of register bit a (a < 5).
constexpr uint32_t kGrpFallback = 1u, kGrpPerm = 1u << 26;
struct UGroup {
    int32_t gidx;       // static group
    int32_t a, b;       // register group: first uop, count; LDS group: op range
    uint32_t flags;
};

__device__ __forceinline__ uint8_t uop_code(const UOp &u)
{
    switch (u.kind) {
    case UK_MAT1: return (uint8_t)(kCodeMat1 + u.j0);
    case UK_MAT1R: return (uint8_t)(kCodeMat1R + u.j0);
    case UK_DIAG1: return (uint8_t)(kCodeDiag1 + u.j0);
    case UK_MAT1M: return (uint8_t)(kCodeMat1M + u.j0);
    case UK_CX: return (uint8_t)(kCodeCX + 6 * u.j0 + u.j1);
    case UK_CZ: return (uint8_t)(kCodeCZ + 6 * u.j0 + u.j1);
    case UK_SWAP: return (uint8_t)(kCodeSwap + 6 * u.j0 + u.j1);
    default: return (uint8_t)kCodeCopy;
    }
}

__device__ __forceinline__ void put_uop(lds<UOp> *p, const UOp &u)
{
    p->kind = u.kind;
    p->j0 = u.j0;
    p->j1 = u.j1;
    p->code = uop_code(u);
    p->mat = u.mat;
    p->pad2 = 0;
}

// Micro-ops are the same for every thread: read them as scalars so that
// their dispatch compiles to scalar branches, not exec-masked compares.
__device__ __forceinline__ uint32_t uni(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float uni(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(uint32_t, v)));
}
__device__ __forceinline__ double uni(double v)
{
    // readfirstlane returns int: go through uint32_t so the low word is not
    // sign-extended into the high word
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)b);
    const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    return __builtin_bit_cast(double, lo | (hi << 32));
}

// Matrix of a one-qubit gate op for the record's shot: a swept U3 takes its
// set's matrix (sets split the run's shots evenly; batch mode, one shot).
__device__ __forceinline__ const double *op_matrix(const ExecParams &P, const DevOp &op,
                                                   const lds<WgShared> &S)
{
    if (!(op.flags & DF_PARAM)) return P.pool + op.mat;
    const uint32_t set = (uint32_t)P.shot_perm[S.lo] / P.shots_per_set;
    return P.pool + op.mat + (size_t)set * P.set_stride;
}

__device__ __forceinline__ UOp get_uop(const lds<UOp> *p)
{
    const uint64_t w = *(const lds<uint64_t> *)p;
    const uint32_t lo = uni((uint32_t)w), hi = uni((uint32_t)(w >> 32));
    UOp u;
    u.kind = (uint8_t)lo;
    u.j0 = (uint8_t)(lo >> 8);
    u.j1 = (uint8_t)(lo >> 16);
    u.code = (uint8_t)(lo >> 24);
    u.mat = (uint16_t)hi;
    u.pad2 = 0;
    return u;
}

// Byte offset of the per-workgroup state in dynamic LDS (after the tile,
// the offset table, the decisions and the micro-op area).
__device__ __forceinline__ uint32_t svb_side_bytes_dev(int tile_q, int amp_bytes, int resident,
                                                      int nbuf)
{
    const uint32_t tile = (1u << tile_q) * amp_bytes * (resident ? 1u : (uint32_t)nbuf);
    const uint32_t hi = resident ? 16u : (1u << (tile_q - kCoalesceQ)) * 4u;
    const uint32_t dec = kMaxPassOps * 2;
    const uint32_t fuse = kMaxPassGroups * (uint32_t)sizeof(UGroup) + kMaxPassUops * (uint32_t)sizeof(UOp) +
                          kPassMatBytes;
    const uint32_t cnt = 16u * kWG * 4u;
    const bool cnt_in_tile = !resident && (1u << tile_q) * amp_bytes >= cnt;
    const uint32_t ua = (!cnt_in_tile && cnt > fuse) ? cnt : fuse;
    return (tile + hi + dec + ua + 15u) / 16u * 16u;
}

// LDS bytes of the op staging area after the per-workgroup state
__host__ __device__ __forceinline__ size_t stage_bytes(int stage_cap)
{
    if (stage_cap <= 0) return 0;
    return (size_t)stage_cap * (sizeof(DevOp) + 8 * sizeof(double)) +
           (kStageRules * sizeof(DevRule) + kStageRules * sizeof(int32_t) + 15) / 16 * 16 +
           2 * kStageTerms * sizeof(double);
}
__host__ __device__ __forceinline__ size_t shared_bytes16()
{
    return (sizeof(WgShared) + 15) / 16 * 16;
}

template <class R>
struct Ctx {
    using A = typename V2<R>::T;
    const ExecParams &P;
    lds<WgShared> &S;
    lds<A> *L;         // LDS tile (2^k amplitudes, swizzled positions)
    uint32_t lbase;    // LDS byte address of L (0, or the second buffer)
    lds<uint32_t> *hi_off;  // LDS: global offset of local index bits >= kCoalesceQ
    lds<int16_t> *dec; // LDS: decided outcome of each op of the pass
    lds<int> *cnt;     // LDS: 16 x kWG outcome counters (splits); aliases the tile
                       // of a streamed state (free between sweeps)
    lds<unsigned char> *scr;  // LDS: scratch (aliases the micro-op area)
    lds<UGroup> *ug;   // LDS: register groups of the pass
    lds<UOp> *uops;    // LDS: micro-ops of the pass
    lds<R> *mats;      // LDS: fused matrices of the pass (8 reals each)
    const DevOp *sops; // staged op records of the pass (LDS, seen through a generic
                       // pointer), or null
    lds<double> *smat; // staged 2x2 matrices (8 doubles) of the staged DK_MAT1 ops
    int s0, scap;      // first staged op, ops staged
    const DevRule *srules;  // staged rule records (generic pointer to LDS), or null
    lds<int32_t> *sroff;    // staged Pauli table offset of each rule
    lds<double> *sthr;      // staged Pauli thresholds, then the term codes
    uint32_t tsize;    // 2^k
    uint32_t n_tiles;  // 2^(n-k), 1 if resident
    uint32_t swm;      // swizzle mask of the current pass (0: identity)
    int k;
    int tid;
    // LDS position of tile index i: bits 6+j and 7+j are added (XOR) to
    // bit j of the low six, for j in swm. Bits 6 and up stay, so the map is
    // its own inverse, and it is linear over GF(2)
    __device__ __forceinline__ uint32_t at(uint32_t i) const
    {
        return i ^ (((i >> 6) ^ (i >> 7)) & swm);
    }
};

// Op record j: from the LDS copy of the pass when staged, else from the
// program in global memory.
template <class R>
__device__ __forceinline__ const DevOp &op_at(const Ctx<R> &c, int j)
{
    const int i = j - c.s0;
    return (i >= 0 && i < c.scap) ? c.sops[i] : c.P.ops[j];
}

// Matrix of one-qubit gate op j (see op_matrix): the staged copy when there is one.
template <class R>
__device__ __forceinline__ const double *op_matrix_at(const Ctx<R> &c, int j, const DevOp &op)
{
    const int i = j - c.s0;
    if (i >= 0 && i < c.scap) return (const double *)(c.smat + (size_t)i * 8);
    return op_matrix(c.P, op, c.S);
}

// Rule r: the LDS copy when the rules are staged.
template <class R>
__device__ __forceinline__ const DevRule &rule_at(const Ctx<R> &c, uint32_t r)
{
    return c.srules ? c.srules[r] : c.P.rules[r];
}

// First Pauli term whose cumulative threshold exceeds u (thresholds from
// LDS when staged).
template <class R>
__device__ __forceinline__ int pauli_pick_c(const Ctx<R> &c, uint32_t r, const DevRule &ru, double u)
{
    const int n = (int)ru.n_terms;
    if (c.srules) {
        const lds<double> *thr = c.sthr + c.sroff[r];
        for (int j = 0; j < n; ++j)
            if (u < thr[j]) return j;
    } else {
        const double *thr = c.P.pool + ru.thr;
        for (int j = 0; j < n; ++j)
            if (u < thr[j]) return j;
    }
    return n - 1;
}

// Term code of drawn term d (see pauli_code), from LDS when staged.
template <class R>
__device__ __forceinline__ uint32_t pauli_code_c(const Ctx<R> &c, uint32_t r, const DevRule &ru, int d)
{
    if (c.srules) return (uint32_t)c.sthr[kStageTerms + c.sroff[r] + d];
    return (uint32_t)c.P.pool[ru.codes + (uint32_t)d];
}

// All threads, once per workgroup: copy the rule records and the Pauli
// thresholds and term codes to LDS (the host stages them only when they
// fit: at most kStageRules rules and kStageTerms Pauli terms).
template <class R>
__device__ __noinline__ void stage_rules(Ctx<R> &c)
{
    const ExecParams &P = c.P;
    if (c.tid == 0) {
        int off = 0;
        for (int r = 0; r < P.n_rules; ++r) {
            c.sroff[r] = off;
            if (!P.rules[r].is_kraus) off += (int)P.rules[r].n_terms;
        }
    }
    constexpr int W = (int)(sizeof(DevRule) / 4);
    const uint32_t *src = (const uint32_t *)P.rules;
    lds<uint32_t> *dst = (lds<uint32_t> *)(lds<DevRule> *)c.srules;
    for (int i = c.tid; i < P.n_rules * W; i += kWG) dst[i] = src[i];
    __syncthreads();
    for (int r = 0; r < P.n_rules; ++r) {
        const DevRule &ru = P.rules[r];
        if (ru.is_kraus) continue;
        const int o = c.sroff[r];
        for (int j = c.tid; j < (int)ru.n_terms; j += kWG) {
            c.sthr[o + j] = P.pool[ru.thr + j];
            c.sthr[kStageTerms + o + j] = P.pool[ru.codes + j];
        }
    }
    __syncthreads();
}

// ----------------------------------------------------------- op sweeps
template <class R>
__device__ void sweep_mat1(Ctx<R> &c, uint32_t b, const Mat2<R> &m, bool diag)
{
    using A = typename V2<R>::T;
    lds<A> *L = c.L;
    if (diag) {
        for (uint32_t i = c.tid; i < c.tsize; i += kWG) {
            const A v = L[c.at(i)];
            L[c.at(i)] = ((i >> b) & 1u) ? cmul<A, R>(m.r[3], m.i[3], v)
                                   : cmul<A, R>(m.r[0], m.i[0], v);
        }
    } else {
        const uint32_t half = c.tsize >> 1, bit = 1u << b;
        for (uint32_t p = c.tid; p < half; p += kWG) {
            const uint32_t i0 = ins0(p, b), i1 = i0 | bit;
            const A a = L[c.at(i0)], d = L[c.at(i1)];
            A o0 = cmul<A, R>(m.r[0], m.i[0], a);
            o0 = cmac<A, R>(o0, m.r[1], m.i[1], d);
            A o1 = cmul<A, R>(m.r[2], m.i[2], a);
            o1 = cmac<A, R>(o1, m.r[3], m.i[3], d);
            L[c.at(i0)] = o0;
            L[c.at(i1)] = o1;
        }
    }
    __syncthreads();
}

// Dense 2^NQ x 2^NQ matrix m (row-major, interleaved re/im doubles, times
// s) on tile bits b[0..NQ-1]; bit t of its row/column index <-> b[t]. Each
// thread owns the 2^NQ amplitudes of one base index: it holds them in
// registers and writes every output row straight back to its own slot.
template <class R, int NQ>
__device__ void sweep_dense_t(Ctx<R> &c, const uint8_t *b, const double *m, double s)
{
    using A = typename V2<R>::T;
    constexpr int D = 1 << NQ;
    uint32_t bits[NQ], sorted[NQ];
#pragma unroll
    for (int t = 0; t < NQ; ++t) bits[t] = sorted[t] = b[t];
    // ascending bit positions for the zero insertion
#pragma unroll
    for (int i = 0; i < NQ; ++i)
#pragma unroll
        for (int j = 0; j + 1 < NQ - i; ++j)
            if (sorted[j] > sorted[j + 1]) {
                const uint32_t t = sorted[j];
                sorted[j] = sorted[j + 1];
                sorted[j + 1] = t;
            }
    lds<A> *L = c.L;
    const uint32_t nbase = c.tsize >> NQ;
    for (uint32_t p = c.tid; p < nbase; p += kWG) {
        uint32_t base = p;
#pragma unroll
        for (int t = 0; t < NQ; ++t) base = ins0(base, sorted[t]);
        A v[D];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            uint32_t idx = base;
#pragma unroll
            for (int t = 0; t < NQ; ++t) idx |= ((uint32_t)(a >> t) & 1u) << bits[t];
            v[a] = L[c.at(idx)];
        }
        for (int a = 0; a < D; ++a) {
            A acc;
            acc.x = 0;
            acc.y = 0;
#pragma unroll
            for (int bb = 0; bb < D; ++bb)
                acc = cmac<A, R>(acc, (R)(m[2 * (a * D + bb)] * s), (R)(m[2 * (a * D + bb) + 1] * s), v[bb]);
            uint32_t idx = base;
#pragma unroll
            for (int t = 0; t < NQ; ++t) idx |= ((uint32_t)(a >> t) & 1u) << bits[t];
            L[c.at(idx)] = acc;
        }
    }
    __syncthreads();
}

template <class R>
__device__ __noinline__ void sweep_dense(Ctx<R> &c, int nq, const uint8_t *b, const double *m,
                                         double s)
{
    switch (nq) {
    case 2: sweep_dense_t<R, 2>(c, b, m, s); break;
    case 3: sweep_dense_t<R, 3>(c, b, m, s); break;
    case 4: sweep_dense_t<R, 4>(c, b, m, s); break;
    default: sweep_dense_t<R, 5>(c, b, m, s); break;
    }
}

template <class R>
__device__ void sweep_cx(Ctx<R> &c, uint32_t bc, uint32_t bt)
{
    using A = typename V2<R>::T;
    const uint32_t lo = bc < bt ? bc : bt, hi = bc < bt ? bt : bc;
    const uint32_t quarter = c.tsize >> 2;
    lds<A> *L = c.L;
    for (uint32_t p = c.tid; p < quarter; p += kWG) {
        const uint32_t i = ins0(ins0(p, lo), hi) | (1u << bc);
        const uint32_t j = i | (1u << bt);
        const A a = L[c.at(i)];
        L[c.at(i)] = L[c.at(j)];
        L[c.at(j)] = a;
    }
    __syncthreads();
}

template <class R>
__device__ void sweep_cz(Ctx<R> &c, uint32_t ba, uint32_t bb)
{
    using A = typename V2<R>::T;
    const uint32_t lo = ba < bb ? ba : bb, hi = ba < bb ? bb : ba;
    const uint32_t quarter = c.tsize >> 2;
    lds<A> *L = c.L;
    for (uint32_t p = c.tid; p < quarter; p += kWG) {
        const uint32_t i = ins0(ins0(p, lo), hi) | (1u << ba) | (1u << bb);
        A a = L[c.at(i)];
        a.x = -a.x;
        a.y = -a.y;
        L[c.at(i)] = a;
    }
    __syncthreads();
}

template <class R>
__device__ void sweep_swap(Ctx<R> &c, uint32_t ba, uint32_t bb)
{
    using A = typename V2<R>::T;
    const uint32_t lo = ba < bb ? ba : bb, hi = ba < bb ? bb : ba;
    const uint32_t quarter = c.tsize >> 2;
    lds<A> *L = c.L;
    for (uint32_t p = c.tid; p < quarter; p += kWG) {
        const uint32_t base = ins0(ins0(p, lo), hi);
        const uint32_t i = base | (1u << ba), j = base | (1u << bb);
        const A a = L[c.at(i)];
        L[c.at(i)] = L[c.at(j)];
        L[c.at(j)] = a;
    }
    __syncthreads();
}

// Pauli string P = (-i)^ny Z^z X^x on local masks (Sec. IV-A, Pauli batching:
// swap of the amplitudes paired by the X/Y mask, phase from the Y count,
// sign from the parity of the destination index under the Z/Y mask).
template <class R>
__device__ void sweep_pauli(Ctx<R> &c, uint32_t xl, uint32_t zl, uint32_t ny)
{
    using A = typename V2<R>::T;
    lds<A> *L = c.L;
    if (xl == 0) {
        for (uint32_t i = c.tid; i < c.tsize; i += kWG)
            L[c.at(i)] = phase_ny(neg_if(L[c.at(i)], __popc(i & zl)), ny);
    } else {
        const uint32_t xb = 31u - __clz(xl);
        const uint32_t half = c.tsize >> 1;
        for (uint32_t p = c.tid; p < half; p += kWG) {
            const uint32_t i0 = ins0(p, xb), i1 = i0 ^ xl;
            const A a = L[c.at(i0)], d = L[c.at(i1)];
            L[c.at(i0)] = phase_ny(neg_if(d, __popc(i0 & zl)), ny);
            L[c.at(i1)] = phase_ny(neg_if(a, __popc(i1 & zl)), ny);
        }
    }
    __syncthreads();
}

// Collapse onto outcome pattern o of the measured local bits, scale by s,
// then (reset) return measured ones to |0>.
template <class R>
__device__ void sweep_measure(Ctx<R> &c, const DevOp &op, uint32_t o, double s)
{
    using A = typename V2<R>::T;
    lds<A> *L = c.L;
    const R sc = (R)s;
    for (uint32_t i = c.tid; i < c.tsize; i += kWG) {
        uint32_t pat = 0;
        for (int t = 0; t < op.nq; ++t) pat |= ((i >> op.lb[t]) & 1u) << t;
        A v = L[c.at(i)];
        if (pat == o) {
            v.x *= sc;
            v.y *= sc;
        } else {
            v.x = 0;
            v.y = 0;
        }
        L[c.at(i)] = v;
    }
    __syncthreads();
    if (op.flags & DF_RESET) {
        for (int t = 0; t < op.nq; ++t) {
            if (!((o >> t) & 1u)) continue;
            const uint32_t b = op.lb[t], half = c.tsize >> 1;
            for (uint32_t p = c.tid; p < half; p += kWG) {
                const uint32_t i0 = ins0(p, b), i1 = i0 | (1u << b);
                const A a = L[c.at(i0)];
                L[c.at(i0)] = L[c.at(i1)];
                L[c.at(i1)] = a;
            }
            __syncthreads();
        }
    }
}

__device__ __forceinline__ uint64_t flops_mat1(bool diag) { return diag ? 6 : 14; }

// Apply op j with decided outcome d (and renormalisation s) to the tile.
template <class R>
__device__ __noinline__ void apply_op(Ctx<R> &c, const DevOp &op, int d, double s)
{
    const ExecParams &P = c.P;
    if (op.kind == DK_BFUNC || ((op.flags & DF_COND) && d == kSkip)) return;
    switch (op.kind) {
    case DK_MAT1: {
        const Mat2<R> m = load_m2<R>(op_matrix(P, op, c.S), 1.0);
        sweep_mat1(c, op.lb[0], m, (op.flags & DF_DIAG) != 0);
        break;
    }
    case DK_MATK:
        sweep_dense(c, op.nq, op.lb, P.pool + op.mat, 1.0);
        break;
    case DK_CX: sweep_cx(c, op.lb[0], op.lb[1]); break;
    case DK_CZ: sweep_cz(c, op.lb[0], op.lb[1]); break;
    case DK_SWAP: sweep_swap(c, op.lb[0], op.lb[1]); break;
    case DK_PAULI: {
        const uint32_t code = pauli_code(P, P.rules[op.rule], d);
        if (code == 0) break;  // identity
        uint32_t xl = 0, zl = 0;
        for (int t = 0; t < op.nq; ++t) {
            xl |= ((code >> t) & 1u) << op.lb[t];
            zl |= ((code >> (8 + t)) & 1u) << op.lb[t];
        }
        sweep_pauli(c, xl, zl, code >> 16);
        break;
    }
    case DK_KRAUS: {
        const DevRule &ru = P.rules[op.rule];
        if (((ru.scalar_mask >> d) & 1u) && s == 1.0) break;  // c * I: norm only
        const uint32_t dim = 1u << ru.nq;
        const double *m = P.pool + ru.mats + (size_t)d * dim * dim * 2;
        if (ru.nq == 1) {
            const Mat2<R> mm = load_m2<R>(m, s);
            const bool diag = m[2] == 0.0 && m[3] == 0.0 && m[4] == 0.0 && m[5] == 0.0;
            sweep_mat1(c, op.lb[0], mm, diag);
        } else {
            sweep_dense(c, (int)ru.nq, op.lb, m, s);
        }
        break;
    }
    case DK_MEASURE:
        sweep_measure(c, op, (uint32_t)d, s);
        break;
    default: break;
    }
}

__device__ __forceinline__ uint64_t op_flops(const ExecParams &P, const DevOp &op, int d)
{
    switch (op.kind) {
    case DK_MAT1: return flops_mat1((op.flags & DF_DIAG) != 0);
    case DK_MATK: return 8ull * (1ull << op.nq) - 2;
    case DK_KRAUS: return 8ull * (1ull << P.rules[op.rule].nq) - 2;
    case DK_MEASURE: return 2;
    default: return 0;
    }
}


// ----------------------------------------------------------- register groups
// In-register ops on a thread's NR amplitudes; J, C, T are register bits.
template <int J, class A, class R, int NR>
__device__ __forceinline__ void r_mat1(A (&v)[NR], const R (&m)[8])
{
    if constexpr ((1 << J) < NR) {
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            if (i & (1 << J)) continue;
            const int i1 = i | (1 << J);
            const A a = v[i], b = v[i1];
            A o0 = cmul<A, R>(m[0], m[1], a);
            o0 = cmac<A, R>(o0, m[2], m[3], b);
            A o1 = cmul<A, R>(m[4], m[5], a);
            o1 = cmac<A, R>(o1, m[6], m[7], b);
            v[i] = o0;
            v[i1] = o1;
        }
    }
}

// Same as r_mat1 for a real top-left entry m[0] (m[1] == 0): the products
// are the ones r_mat1 forms, without the terms that multiply by zero.
template <int J, class A, class R, int NR>
__device__ __forceinline__ void r_mat1r(A (&v)[NR], const R (&m)[8])
{
    if constexpr ((1 << J) < NR) {
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            if (i & (1 << J)) continue;
            const int i1 = i | (1 << J);
            const A a = v[i], b = v[i1];
            A o0;
            o0.x = m[0] * a.x;
            o0.y = m[0] * a.y;
            o0 = cmac<A, R>(o0, m[2], m[3], b);
            A o1 = cmul<A, R>(m[4], m[5], a);
            o1 = cmac<A, R>(o1, m[6], m[7], b);
            v[i] = o0;
            v[i1] = o1;
        }
    }
}

template <int J, class A, class R, int NR>
__device__ __forceinline__ void r_diag1(A (&v)[NR], const R (&m)[8])
{
    if constexpr ((1 << J) < NR) {
#pragma unroll
        for (int i = 0; i < NR; ++i)
            v[i] = (i & (1 << J)) ? cmul<A, R>(m[6], m[7], v[i]) : cmul<A, R>(m[0], m[1], v[i]);
    }
}

template <int C, int T, class A, int NR>
__device__ __forceinline__ void r_cx(A (&v)[NR])
{
    if constexpr ((1 << C) < NR && (1 << T) < NR && C != T) {
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            if (!(i & (1 << C)) || (i & (1 << T))) continue;
            const A a = v[i];
            v[i] = v[i | (1 << T)];
            v[i | (1 << T)] = a;
        }
    }
}

template <int C, int T, class A, int NR>
__device__ __forceinline__ void r_cz(A (&v)[NR])
{
    if constexpr ((1 << C) < NR && (1 << T) < NR && C != T) {
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            if ((i & (1 << C)) && (i & (1 << T))) {
                v[i].x = -v[i].x;
                v[i].y = -v[i].y;
            }
        }
    }
}

template <int C, int T, class A, int NR>
__device__ __forceinline__ void r_swap(A (&v)[NR])
{
    if constexpr ((1 << C) < NR && (1 << T) < NR && C != T) {
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            if (!(i & (1 << C)) || (i & (1 << T))) continue;
            const int i2 = (i ^ (1 << C)) | (1 << T);
            const A a = v[i];
            v[i] = v[i2];
            v[i2] = a;
        }
    }
}

template <class A, class R, int NR>
__device__ __forceinline__ void d_mat1(A (&v)[NR], int j, const R (&m)[8], int kind)
{
#define SVB_M1(J)                                   \
    case J:                                         \
        if (kind == UK_MAT1R) r_mat1r<J, A, R, NR>(v, m);  \
        else if (kind == UK_DIAG1) r_diag1<J, A, R, NR>(v, m); \
        else r_mat1<J, A, R, NR>(v, m);             \
        break;
    switch (j) { SVB_M1(0) SVB_M1(1) SVB_M1(2) SVB_M1(3) SVB_M1(4) SVB_M1(5) default: break; }
#undef SVB_M1
}

// complex64 one-qubit micro-op on the matrix cores. A 2x2 complex matrix
// acting on an amplitude pair (a, b) is the real 4x4 matrix M acting on
// x = (re a, im a, re b, im b). v_mfma_f32_4x4x1f32 (16 blocks of 4 lanes)
// computes, in lane l and result register i, sum over its K = 1 of
// A(lane 4*(l/4) + i) * B(lane l). With lane l holding row l%4 of column k
// of M in A and component k of its own pair in B, four accumulating
// instructions give each lane M x for its pair: the same 16 products per
// pair as the vector form, off the vector ALU (measured in registers on
// gfx950: 1.23x the vector form's rate per gate).
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int J, int NR>
__device__ __forceinline__ void r_mat1_mfma(f32x2 (&v)[NR], const float (&a)[4])
{
    if constexpr ((1 << J) < NR) {
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            if (i & (1 << J)) continue;
            const int i1 = i | (1 << J);
            f32x4 d = {0.f, 0.f, 0.f, 0.f};
            d = __builtin_amdgcn_mfma_f32_4x4x1f32(a[0], v[i].x, d, 0, 0, 0);
            d = __builtin_amdgcn_mfma_f32_4x4x1f32(a[1], v[i].y, d, 0, 0, 0);
            d = __builtin_amdgcn_mfma_f32_4x4x1f32(a[2], v[i1].x, d, 0, 0, 0);
            d = __builtin_amdgcn_mfma_f32_4x4x1f32(a[3], v[i1].y, d, 0, 0, 0);
            v[i].x = d[0];
            v[i].y = d[1];
            v[i1].x = d[2];
            v[i1].y = d[3];
        }
    }
}

template <int NR>
__device__ __forceinline__ void d_mat1_mfma(f32x2 (&v)[NR], int j, const float (&a)[4])
{
#define SVB_M1(J) case J: r_mat1_mfma<J, NR>(v, a); break;
    switch (j) { SVB_M1(0) SVB_M1(1) SVB_M1(2) SVB_M1(3) SVB_M1(4) SVB_M1(5) default: break; }
#undef SVB_M1
}

// This lane's entries of the real 4x4 form of the fused matrix m (row-major
// 2x2 complex, interleaved re/im): row r = lane % 4 of columns 0..3.
//   r = 0: ( re m00, -im m00,  re m01, -im m01)    (re of output a)
//   r = 1: ( im m00,  re m00,  im m01,  re m01)    (im of output a)
//   r = 2, 3: the same with m10, m11               (output b)
__device__ __forceinline__ void mfma_rows(const lds<float> *m, uint32_t lane, float (&a)[4])
{
    const uint32_t r = lane & 3u;
    const f32x4 x = *(const lds<f32x4> *)(m + (r >> 1) * 4);
    const bool odd = (r & 1u) != 0;
    a[0] = odd ? x.y : x.x;
    a[1] = odd ? x.x : -x.y;
    a[2] = odd ? x.w : x.z;
    a[3] = odd ? x.z : -x.w;
}

template <class A, int NR>
__device__ __forceinline__ void d_two(A (&v)[NR], int kind, int c, int t)
{
#define SVB_P(C, T)                                        \
    case C * 8 + T:                                        \
        if (kind == UK_CX) r_cx<C, T, A, NR>(v);           \
        else if (kind == UK_CZ) r_cz<C, T, A, NR>(v);      \
        else r_swap<C, T, A, NR>(v);                       \
        break;
#define SVB_ROW(C) SVB_P(C, 0) SVB_P(C, 1) SVB_P(C, 2) SVB_P(C, 3) SVB_P(C, 4) SVB_P(C, 5)
    switch (c * 8 + t) { SVB_ROW(0) SVB_ROW(1) SVB_ROW(2) SVB_ROW(3) SVB_ROW(4) SVB_ROW(5) default: break; }
#undef SVB_ROW
#undef SVB_P
}

// ---- two register sets: a micro-op reads one and writes every entry of
// the other, so a one-qubit micro-op needs no copies; the register-group
// loop alternates between the two sets (micro-op counts are padded to even)
template <class A, int NR>
__device__ __forceinline__ void p_copy(const A (&v)[NR], A (&o)[NR])
{
#pragma unroll
    for (int i = 0; i < NR; ++i) o[i] = v[i];
}

template <int J, class A, class R, int NR>
__device__ __forceinline__ void p_mat1(const A (&v)[NR], A (&o)[NR], const R (&m)[8])
{
    if constexpr ((1 << J) < NR) {
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            if (i & (1 << J)) continue;
            const int i1 = i | (1 << J);
            const A a = v[i], b = v[i1];
            A o0 = cmul<A, R>(m[0], m[1], a);
            o0 = cmac<A, R>(o0, m[2], m[3], b);
            A o1 = cmul<A, R>(m[4], m[5], a);
            o1 = cmac<A, R>(o1, m[6], m[7], b);
            o[i] = o0;
            o[i1] = o1;
        }
    } else {
        p_copy<A, NR>(v, o);
    }
}

// real top-left entry m[0] (m[1] == 0)
template <int J, class A, class R, int NR>
__device__ __forceinline__ void p_mat1r(const A (&v)[NR], A (&o)[NR], const R (&m)[8])
{
    if constexpr ((1 << J) < NR) {
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            if (i & (1 << J)) continue;
            const int i1 = i | (1 << J);
            const A a = v[i], b = v[i1];
            A o0;
            o0.x = m[0] * a.x;
            o0.y = m[0] * a.y;
            o0 = cmac<A, R>(o0, m[2], m[3], b);
            A o1 = cmul<A, R>(m[4], m[5], a);
            o1 = cmac<A, R>(o1, m[6], m[7], b);
            o[i] = o0;
            o[i1] = o1;
        }
    } else {
        p_copy<A, NR>(v, o);
    }
}

template <int J, class A, class R, int NR>
__device__ __forceinline__ void p_diag1(const A (&v)[NR], A (&o)[NR], const R (&m)[8])
{
    if constexpr ((1 << J) < NR) {
#pragma unroll
        for (int i = 0; i < NR; ++i)
            o[i] = (i & (1 << J)) ? cmul<A, R>(m[6], m[7], v[i]) : cmul<A, R>(m[0], m[1], v[i]);
    } else {
        p_copy<A, NR>(v, o);
    }
}

template <int C, int T, class A, int NR>
__device__ __forceinline__ void p_cx(const A (&v)[NR], A (&o)[NR])
{
    if constexpr ((1 << C) < NR && (1 << T) < NR && C != T) {
#pragma unroll
        for (int i = 0; i < NR; ++i) o[i] = v[(i & (1 << C)) ? (i ^ (1 << T)) : i];
    } else {
        p_copy<A, NR>(v, o);
    }
}

template <int C, int T, class A, int NR>
__device__ __forceinline__ void p_cz(const A (&v)[NR], A (&o)[NR])
{
    if constexpr ((1 << C) < NR && (1 << T) < NR && C != T) {
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            o[i] = v[i];
            if ((i & (1 << C)) && (i & (1 << T))) {
                o[i].x = -v[i].x;
                o[i].y = -v[i].y;
            }
        }
    } else {
        p_copy<A, NR>(v, o);
    }
}

template <int C, int T, class A, int NR>
__device__ __forceinline__ void p_swap(const A (&v)[NR], A (&o)[NR])
{
    if constexpr ((1 << C) < NR && (1 << T) < NR && C != T) {
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            const int bc = (i >> C) & 1, bt = (i >> T) & 1;
            o[i] = v[(i & ~((1 << C) | (1 << T))) | (bc << T) | (bt << C)];
        }
    } else {
        p_copy<A, NR>(v, o);
    }
}


// Matrix-core one-qubit micro-op on two register sets: out = M in for
// every pair on register bit J (see r_mat1_mfma for the lane layout).
template <int J, int NR>
__device__ __forceinline__ void p_mat1_mfma(const f32x2 (&v)[NR], f32x2 (&o)[NR], const float (&a)[4])
{
    if constexpr ((1 << J) < NR) {
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            if (i & (1 << J)) continue;
            const int i1 = i | (1 << J);
            f32x4 d = {0.f, 0.f, 0.f, 0.f};
            d = __builtin_amdgcn_mfma_f32_4x4x1f32(a[0], v[i].x, d, 0, 0, 0);
            d = __builtin_amdgcn_mfma_f32_4x4x1f32(a[1], v[i].y, d, 0, 0, 0);
            d = __builtin_amdgcn_mfma_f32_4x4x1f32(a[2], v[i1].x, d, 0, 0, 0);
            d = __builtin_amdgcn_mfma_f32_4x4x1f32(a[3], v[i1].y, d, 0, 0, 0);
            o[i].x = d[0];
            o[i].y = d[1];
            o[i1].x = d[2];
            o[i1].y = d[3];
        }
    } else {
        p_copy<f32x2, NR>(v, o);
    }
}

// out = micro-op u applied to in (every entry of out written)
template <class R, int NR, bool MF>
__device__ __forceinline__ void apply_uop(const typename V2<R>::T (&in)[NR],
                                          typename V2<R>::T (&out)[NR], const UOp &u,
                                          const lds<R> *mats, int tid)
{
    using A = typename V2<R>::T;
    const uint32_t code = u.code;
    if (code < kCodeCX) {
        R m[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) m[e] = uni(mats[u.mat * 8 + e]);
#define SVB_P1(J)                                                        \
    case kCodeMat1 + J: p_mat1<J, A, R, NR>(in, out, m); break;          \
    case kCodeMat1R + J: p_mat1r<J, A, R, NR>(in, out, m); break;        \
    case kCodeDiag1 + J: p_diag1<J, A, R, NR>(in, out, m); break;
        switch (code) { SVB_P1(0) SVB_P1(1) SVB_P1(2) SVB_P1(3) SVB_P1(4) SVB_P1(5) default: p_copy<A, NR>(in, out); }
#undef SVB_P1
    } else if (MF && code >= kCodeMat1M && code < kCodeMat1M + 6) {
        if constexpr (MF && sizeof(R) == 4) {
            float a4[4];
            mfma_rows(mats + u.mat * 8, (uint32_t)tid, a4);
#define SVB_PM(J) case kCodeMat1M + J: p_mat1_mfma<J, NR>(in, out, a4); break;
            switch (code) { SVB_PM(0) SVB_PM(1) SVB_PM(2) SVB_PM(3) SVB_PM(4) SVB_PM(5) default: p_copy<A, NR>(in, out); }
#undef SVB_PM
        } else {
            p_copy<A, NR>(in, out);
        }
    } else {
#define SVB_P2(C, T)                                                     \
    case kCodeCX + 6 * C + T: p_cx<C, T, A, NR>(in, out); break;         \
    case kCodeCZ + 6 * C + T: p_cz<C, T, A, NR>(in, out); break;         \
    case kCodeSwap + 6 * C + T: p_swap<C, T, A, NR>(in, out); break;
#define SVB_P2ROW(C) SVB_P2(C, 0) SVB_P2(C, 1) SVB_P2(C, 2) SVB_P2(C, 3) SVB_P2(C, 4) SVB_P2(C, 5)
        switch (code) { SVB_P2ROW(0) SVB_P2ROW(1) SVB_P2ROW(2) SVB_P2ROW(3) SVB_P2ROW(4) SVB_P2ROW(5)
                        default: p_copy<A, NR>(in, out); }
#undef SVB_P2ROW
#undef SVB_P2
    }
}

// Register groups whose two register sets fit the budget of two
// workgroups per compute unit run the alternating form; larger ones
// (64 complex64 or 32 complex128 amplitudes per thread) update one set
template <class R, int NR>
constexpr bool two_sets() { return NR * (int)sizeof(typename V2<R>::T) <= 256; }

// Values the tile loop needs, held in registers: the executor context
// lives in private memory (cold paths take it by reference), and a private
// load inside the loop would wait for the tile copies in flight.
struct Hot {
    uint32_t ug, uops, mats;  // LDS byte addresses of the pass's groups, micro-ops, matrices
    uint32_t lbase;           // LDS byte address of the current tile buffer
    uint32_t hi;              // LDS byte address of the tile's global-offset table
    uint32_t swm;             // swizzle mask
    int n_ug, k, tid;
    __device__ __forceinline__ uint32_t at(uint32_t i) const
    {
        return i ^ (((i >> 6) ^ (i >> 7)) & swm);
    }
};

template <class R, int NR> struct Direct;

// Gather the thread's NR amplitudes of group gi from LDS, run the group's
// micro-ops in registers, scatter back (to LDS, or with DIRECT to HBM).
template <class R, int NR, bool MF>
__device__ __forceinline__ void run_group(const Hot &h, const cst<GroupInfo> &gi, int first, int count,
                                          uint32_t gfl, bool direct, const Direct<R, NR> &d)
{
    using A = typename V2<R>::T;
    constexpr int RB = NR >= 64 ? 6 : NR >= 32 ? 5 : NR >= 16 ? 4 : NR >= 8 ? 3 : 2;
    constexpr int SH = sizeof(A) == 8 ? 3 : 4;
    // scalar loads are whole dwords: read the position bytes as words
    const cst<uint32_t> *gw = (const cst<uint32_t> *)&gi;
    uint32_t gpw[2], cpw[4];
#pragma unroll
    for (int i = 0; i < 2; ++i) gpw[i] = gw[offsetof(GroupInfo, gpos) / 4 + i];
#pragma unroll
    for (int i = 0; i < 4; ++i) cpw[i] = gw[offsetof(GroupInfo, cpos) / 4 + i];
    uint32_t base = 0;
    for (int i = 0; i < h.k - RB; ++i)
        base |= ((uint32_t)(h.tid >> i) & 1u) << ((cpw[i >> 2] >> (8 * (i & 3))) & 0xffu);
    // byte position of register i = (thread part) ^ (uniform part); the
    // swizzle is linear over disjoint bits, so the parts combine by XOR.
    // A second tile buffer starts at the tile size, a power of two above
    // every in-tile byte position, so OR-ing its base commutes with the XORs
    const uint32_t pb8 = (h.at(base) << SH) | h.lbase;
    uint32_t pe8[RB];
#pragma unroll
    for (int j = 0; j < RB; ++j)
        pe8[j] = __builtin_amdgcn_readfirstlane(h.at(1u << ((gpw[j >> 2] >> (8 * (j & 3))) & 0xffu)) << SH);
    uint32_t K[NR];
    K[0] = 0;
#pragma unroll
    for (int i = 1; i < NR; ++i) K[i] = K[i & (i - 1)] ^ pe8[__builtin_ctz(i)];
    // pb8 ^ K[i] is the LDS address itself
    A v[NR];
#pragma unroll
    for (int i = 0; i < NR; ++i) v[i] = *(const lds<A> *)(size_t)(pb8 ^ K[i]);
    if (direct) {
        lds_sync();  // every thread has its amplitudes: the buffer is free
        if (d.issue_next) d.io.issue(d.state, d.next_base, 0);
    }
    const lds<UOp> *uops = (const lds<UOp> *)(size_t)h.uops;
    const lds<R> *mats = (const lds<R> *)(size_t)h.mats;
    // image of register bit a under the group's closing permutation (the
    // identity unless the flags carry one)
    uint32_t img[RB];
#pragma unroll
    for (int a = 0; a < RB; ++a) img[a] = 1u << a;
    if constexpr (two_sets<R, NR>()) {
        A w[NR];
        for (int q = 0; q < count; q += 2) {  // count is even
            apply_uop<R, NR, MF>(v, w, get_uop(uops + first + q), mats, h.tid);
            apply_uop<R, NR, MF>(w, v, get_uop(uops + first + q + 1), mats, h.tid);
        }
        if (gfl & kGrpPerm) {
#pragma unroll
            for (int a = 0; a < RB; ++a) img[a] = (gfl >> (1 + 5 * a)) & 31u;
        }
    } else {
        for (int q = 0; q < count; ++q) {
            const UOp u = get_uop(uops + first + q);
            if (u.code == kCodeCopy) continue;
            if (u.kind == UK_MAT1 || u.kind == UK_DIAG1 || u.kind == UK_MAT1R || u.kind == UK_MAT1M) {
                if constexpr (sizeof(R) == 4) {
                    float a4[4];
                    mfma_rows(mats + u.mat * 8, (uint32_t)h.tid, a4);
                    d_mat1_mfma<NR>(v, u.j0, a4);
                } else {
                    R m[8];
#pragma unroll
                    for (int e = 0; e < 8; ++e) m[e] = uni(mats[u.mat * 8 + e]);
                    d_mat1<A, R, NR>(v, u.j0, m, u.kind);
                }
            } else {
                d_two<A, NR>(v, u.kind, u.j0, u.j1);
            }
        }
    }
    // register i holds group index i; it is stored at the position of the
    // permuted index: XOR over the set bits a of i of the images img[a].
    // One copy of the group body serves both stores (a smaller hot loop)
    if (direct) {
        // global amplitude offset of tile index x: hi[x >> kCoalesceQ] + (x & kRunMask),
        // a bit deposit (register bits and thread bits land on distinct
        // bits, so parts combine by XOR or addition alike)
        const lds<uint32_t> *hi = (const lds<uint32_t> *)(size_t)h.hi;
        const uint32_t gbase = hi[base >> kCoalesceQ] + (base & kRunMask);
        uint32_t ge[RB];
#pragma unroll
        for (int j = 0; j < RB; ++j) {
            const uint32_t x = 1u << ((gpw[j >> 2] >> (8 * (j & 3))) & 0xffu);
            ge[j] = __builtin_amdgcn_readfirstlane(hi[x >> kCoalesceQ] + (x & kRunMask));
        }
        uint32_t gi8[RB];
#pragma unroll
        for (int a = 0; a < RB; ++a) {
            uint32_t g = 0;
#pragma unroll
            for (int b = 0; b < RB; ++b)
                if ((img[a] >> b) & 1u) g ^= ge[b];
            gi8[a] = g;
        }
        // uniform part in the scalar base, thread part as the 32-bit vector
        // offset: one address register for all NR stores
        const uint32_t voff = gbase * (uint32_t)sizeof(A);
        uint32_t G[NR];
        G[0] = 0;
#pragma unroll
        for (int i = 1; i < NR; ++i) G[i] = G[i & (i - 1)] ^ gi8[__builtin_ctz(i)];
        gbl<A> *const tile = uni_ptr(d.tile);
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            gbl<unsigned char> *sb = (gbl<unsigned char> *)(tile + G[i]);
            *(gbl<A> *)(sb + voff) = v[i];
        }
    } else {
        uint32_t pi8[RB];
#pragma unroll
        for (int a = 0; a < RB; ++a) {
            uint32_t p = 0;
#pragma unroll
            for (int b = 0; b < RB; ++b)
                if ((img[a] >> b) & 1u) p ^= pe8[b];
            pi8[a] = p;
        }
        uint32_t K2[NR];
        K2[0] = 0;
#pragma unroll
        for (int i = 1; i < NR; ++i) K2[i] = K2[i & (i - 1)] ^ pi8[__builtin_ctz(i)];
        // recompute the addresses rather than keep NR of them live
        uint32_t pw = pb8;
        asm volatile("" : "+v"(pw));
#pragma unroll
        for (int i = 0; i < NR; ++i) *(lds<A> *)(size_t)(pw ^ K2[i]) = v[i];
        lds_sync();
    }
}

// Per-pass chunk offsets of a thread for streamed tile copies: global byte
// offset from the tile's base (uniform) and LDS byte position, so a copy
// is a scalar-base load/store with a precomputed vector offset.
template <class R, int NR>
struct TileIO {
    // Copy chunk u of thread t is LDS byte (u*kWG + t)*16 of a tile buffer.
    // Its global offset (hi_off is a bit deposit, the swizzle an XOR of bit
    // fields) splits into a per-thread part and a per-u part that is the
    // same for every thread of the workgroup.
    using A = typename V2<R>::T;
    static constexpr int V = 16 / sizeof(A);
    static constexpr int NC = NR / V;
    static constexpr int LNC = NC >= 64 ? 6 : NC >= 32 ? 5 : NC >= 16 ? 4 : NC >= 8 ? 3 : NC >= 4 ? 2 : NC >= 2 ? 1 : 0;
    // LDS is filled and drained in linear order (16 bytes per lane, a wave
    // covers 1 KB), so a tile is fetched straight into LDS with no register
    // staging. LDS byte (u*kWG + t)*16 of a buffer holds tile index at(p),
    // p = (u*kWG + t)*V; at() is its own inverse, so the amplitude of tile
    // index l sits at position at(l), where the register groups expect it.
    // Global offsets are kept in 16-byte chunks (the size of one copy), so
    // 32 bits reach every byte of a state of up to 64 GiB.
    uint32_t lt;          // per-thread global chunk offset of linear chunk 0
    uint32_t lb[LNC + 1]; // global chunk offset of linear chunk-index bit j (uniform)
    uint32_t tid;

    __device__ void setup_linear(Ctx<R> &c)
    {
        tid = (uint32_t)c.tid;
        const uint32_t l = c.at((uint32_t)c.tid * V);
        lt = (c.hi_off[l >> kCoalesceQ] + (l & kRunMask)) / V;
#pragma unroll
        for (int j = 0; j < LNC; ++j) {
            const uint32_t m = c.at((uint32_t)((kWG * V) << j));
            lb[j] = __builtin_amdgcn_readfirstlane((c.hi_off[m >> kCoalesceQ] + (m & kRunMask)) / V);
        }
    }
    __device__ __forceinline__ uint32_t lu(int u) const
    {
        uint32_t g = 0;
#pragma unroll
        for (int j = 0; j < LNC; ++j)
            if (u & (1 << j)) g ^= lb[j];
        return g;
    }
    // Issue the asynchronous global->LDS copy of the tile at base into the
    // buffer at LDS byte address buf; complete after wait_vm() + barrier.
    __device__ void issue(const gbl<A> *Gt, uint64_t base, uint32_t buf) const
    {
        const gbl<u32x4> *G16 = (const gbl<u32x4> *)(Gt + base);
        const uint32_t wb = __builtin_amdgcn_readfirstlane(buf + (tid & ~63u) * 16u);
#pragma unroll
        for (int u = 0; u < NC; ++u)
            __builtin_amdgcn_global_load_lds((const gbl<void> *)(G16 + (lt ^ lu(u))),
                                             (lds<void> *)(size_t)(wb + (uint32_t)u * kWG * 16u),
                                             16, 0, 0);
    }
    // The tile of the virtual |0..0> state: zeros, and amplitude 1 at tile
    // index 0 (LDS position 0) of the tile that holds global index 0.
    __device__ void zero(bool holds_origin) const
    {
        const uint32_t p0 = tid * 16u;
        u32x4 z = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int u = 0; u < NC; ++u) *(lds<u32x4> *)(size_t)(p0 + (uint32_t)u * kWG * 16u) = z;
        if (holds_origin && tid == 0) {
            A one;
            one.x = (R)1;
            one.y = (R)0;
            *(lds<A> *)(size_t)0 = one;
        }
    }
    __device__ void store_linear(gbl<A> *Gt, uint64_t base, uint32_t buf) const
    {
        gbl<u32x4> *G16 = (gbl<u32x4> *)(Gt + base);
        const uint32_t p0 = buf + tid * 16u;
#pragma unroll
        for (int u = 0; u < NC; ++u)
            G16[lt ^ lu(u)] =
                *(const lds<u32x4> *)(size_t)(p0 + (uint32_t)u * kWG * 16u);
    }

};

// The last register group of a tile may write its results straight from
// registers to the state in HBM. The tile buffer is then free once the
// group has gathered, and the next tile's copy into it is issued before
// the group computes. Passed by value through inlined code: nothing here
// may live in private memory.
template <class R, int NR>
struct Direct {
    gbl<typename V2<R>::T> *tile;  // the state at this tile's base
    const gbl<typename V2<R>::T> *state;
    uint64_t next_base;            // the next tile's base, if issue_next
    bool issue_next;
    TileIO<R, NR> io;
};

// ---- plan-time fusion: per register bit a pending FP64 2x2 matrix
// collects consecutive one-qubit factors (gate, drawn Pauli, chosen Kraus
// matrix); two-qubit permutations flush the pending factors of their bits
// and are emitted as they are. Register groups are independent, so each
// group is fused by its own lane of the first wave, with its pending
// matrices in that lane's registers.
constexpr int kMaxRegBits = 6;  // register bits of a group (64 amplitudes per thread)

struct PendRegs {
    double m[kMaxRegBits][8];  // row-major 2x2, interleaved re/im
    uint32_t set;              // bit j: m[j] holds a pending product
};

__device__ __forceinline__ void m2_mul_left(double (&pm)[8], const double (&a)[8])
{
    // pm <- a * pm
    double o[8];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int cc = 0; cc < 2; ++cc) {
            double re = 0, im = 0;
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const double ar = a[2 * (2 * r + t)], ai = a[2 * (2 * r + t) + 1];
                const double br = pm[2 * (2 * t + cc)], bi = pm[2 * (2 * t + cc) + 1];
                re += ar * br - ai * bi;
                im += ar * bi + ai * br;
            }
            o[2 * (2 * r + cc)] = re;
            o[2 * (2 * r + cc) + 1] = im;
        }
#pragma unroll
    for (int e = 0; e < 8; ++e) pm[e] = o[e];
}

// Multiply factor m * scale into the pending matrix of register bit j.
__device__ __forceinline__ void fuse_factor(PendRegs &p, int j, const double *m, double scale)
{
    double a[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) a[e] = m[e] * scale;
    if ((p.set >> j) & 1u) {
        m2_mul_left(p.m[j], a);
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) p.m[j][e] = a[e];
    }
    p.set |= 1u << j;
}

// Emit the pending matrix of bit j (if any) as a one-qubit micro-op (mf: a
// non-diagonal one for the matrix cores). Writes stay below the group's
// micro-op and matrix limits ul, ml; the counts nu, nm advance regardless,
// so an overrun shows in them.
template <class R>
__device__ __forceinline__ void fuse_flush(Ctx<R> &c, PendRegs &p, int j, int &nu, int &nm, int ul,
                                           int ml, uint64_t &flops, bool mf)
{
    if (!((p.set >> j) & 1u)) return;
    p.set &= ~(1u << j);
    double pm[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) pm[e] = p.m[j][e];
    const bool diag = pm[2] == 0.0 && pm[3] == 0.0 && pm[4] == 0.0 && pm[5] == 0.0;
    if (nm < ml) {
#pragma unroll
        for (int e = 0; e < 8; ++e) c.mats[nm * 8 + e] = (R)pm[e];
    }
    UOp u;
    u.kind = diag ? UK_DIAG1 : mf ? UK_MAT1M : (pm[1] == 0.0 ? UK_MAT1R : UK_MAT1);
    u.j0 = (uint8_t)j;
    u.j1 = 0;
    u.code = 0;
    u.mat = (uint16_t)nm;
    u.pad2 = 0;
    if (nu < ul) put_uop(c.uops + nu, u);
    ++nu;
    ++nm;
    flops += diag ? 6 : (pm[1] == 0.0 ? 12 : 14);
}

// The lane that built a group, after its micro-ops [first, nu) are built. CX and SWAP
// micro-ops that commute with every later micro-op of the group (no later
// micro-op touches their register bits) move to the end, in order, and are
// taken out: their product P is a permutation of the register index that
// the group applies by storing register i at the position of P(i). The
// remaining count is padded to even with a copy. Returns the group flags.
__device__ __forceinline__ UOp read_uop(const lds<UOp> *p)
{
    UOp u;
    u.kind = p->kind;
    u.j0 = p->j0;
    u.j1 = p->j1;
    u.code = p->code;
    u.mat = p->mat;
    u.pad2 = 0;
    return u;
}

__device__ uint32_t fold_trailing_perms(lds<UOp> *u, int first, int &nu)
{
    const int cnt = nu - first;
    const int lo = cnt > 64 ? cnt - 64 : 0;
    uint64_t folded = 0;
    uint32_t later = 0;  // register bits of the kept micro-ops after position i
    for (int i = cnt - 1; i >= lo; --i) {
        const UOp x = read_uop(u + first + i);
        if (x.code == kCodeCopy) continue;
        const bool two = x.kind == UK_CX || x.kind == UK_CZ || x.kind == UK_SWAP;
        const uint32_t bits = (1u << x.j0) | (two ? (1u << x.j1) : 0u);
        if ((x.kind == UK_CX || x.kind == UK_SWAP) && !(bits & later)) {
            folded |= 1ull << (i - lo);
            continue;
        }
        later |= bits;
    }
    uint32_t img[5] = {1u, 2u, 4u, 8u, 16u};
    int kept = first;
    for (int i = 0; i < cnt; ++i) {
        const UOp x = read_uop(u + first + i);
        if (i >= lo && ((folded >> (i - lo)) & 1ull)) {
            for (int a = 0; a < 5; ++a) {
                const uint32_t bc = (img[a] >> x.j0) & 1u, bt = (img[a] >> x.j1) & 1u;
                if (x.kind == UK_CX) {
                    img[a] ^= bc << x.j1;
                } else {
                    img[a] = (img[a] & ~((1u << x.j0) | (1u << x.j1))) | (bc << x.j1) | (bt << x.j0);
                }
            }
            continue;
        }
        if (x.code == kCodeCopy) continue;
        put_uop(u + kept++, x);
    }
    nu = kept;
    if ((nu - first) & 1) {
        UOp cp;
        cp.kind = 0;
        cp.j0 = 0;
        cp.j1 = 0;
        cp.code = (uint8_t)kCodeCopy;
        cp.mat = 0;
        cp.pad2 = 0;
        put_uop(u + nu++, cp);
    }
    if (!folded) return 0u;
    uint32_t f = kGrpPerm;
    for (int a = 0; a < 5; ++a) f |= img[a] << (1 + 5 * a);
    return f;
}

// Micro-ops and matrices that ops [a, b) of a register group produce
// before trailing permutations are folded: they follow from the op kinds,
// register bits and decisions alone. Stops before the first op o at which
// fewer than 12 micro-op slots (the op's three, a final flush of eight and
// an even-count pad) or 11 matrix slots remain of room_u, room_m; returns
// the op it stopped at (b if none).
template <class R>
__device__ int group_shape(const Ctx<R> &c, int a, int b, int room_u, int room_m, int &nu, int &nm)
{
    const ExecParams &P = c.P;
    const lds<WgShared> &S = c.S;
    uint32_t pend = 0;
    nu = 0;
    nm = 0;
    int o = a;
    for (; o < b; ++o) {
        if (nu + 12 > room_u || nm + 11 > room_m) break;
        const DevOp &op = op_at(c, o);
        const int d = c.dec[o - S.start];
        const double sc = (o == S.start && S.pending >= 0) ? S.first_scale : 1.0;
        if (op.kind == DK_BFUNC || ((op.flags & DF_COND) && d == kSkip)) continue;
        switch (op.kind) {
        case DK_MAT1:
            pend |= 1u << op.rb[0];
            break;
        case DK_KRAUS: {
            const DevRule &ru = rule_at(c, op.rule);
            if (((ru.scalar_mask >> d) & 1u) && sc == 1.0) break;
            pend |= 1u << op.rb[0];
            break;
        }
        case DK_PAULI: {
            const uint32_t code = pauli_code_c(c, op.rule, rule_at(c, op.rule), d);
            for (int t = 0; t < op.nq; ++t)
                if (((code >> t) | (code >> (8 + t))) & 1u) pend |= 1u << op.rb[t];
            break;
        }
        default: {  // CX, CZ, SWAP: flush both bits, then the micro-op itself
            const uint32_t f = pend & ((1u << op.rb[0]) | (1u << op.rb[1]));
            nu += __builtin_popcount(f) + 1;
            nm += __builtin_popcount(f);
            pend &= ~f;
        }
        }
    }
    (void)P;
    nu += __builtin_popcount(pend);
    nm += __builtin_popcount(pend);
    return o;
}

// Build the register groups and micro-ops of [S.start, S.end) with the
// pass's decisions; may shorten the pass if LDS room runs out. Called by
// every thread (the first wave does the work); ends with a barrier.
//  1. Group boundaries: the static group changes between consecutive ops.
//  2. Each lane counts its group's micro-ops and matrices; exclusive scans
//     give every group its own micro-op and matrix range. The first group
//     that does not fit is cut (or dropped) and ends the pass.
//  3. Each lane fuses its group into its range and folds its trailing
//     permutations.
template <class R>
__device__ __noinline__ void build_uops(Ctx<R> &c)
{
    const ExecParams &P = c.P;
    lds<WgShared> &S = c.S;
    const int tid = c.tid;
    const int start = S.start, end0 = S.end;
    constexpr int kMats = kPassMatBytes / (8 * (int)sizeof(R));
    static_assert(kMaxPassGroups <= 64, "one lane of the first wave per group");
    // groups that run on two register sets (see two_sets): closing
    // permutations are folded into the stores, counts padded to even
    const bool pairs = (1u << (P.tile_q - kWGBits)) * sizeof(typename V2<R>::T) <= 256u;
    const bool mf = sizeof(R) == 4 && P.mfma1 != 0;  // read once, not after every LDS store
    int ng = 0, end = end0;
    if (tid < 64) {
        for (int base = start; base < end0; base += 64) {
            const int o = base + tid;
            const bool in = o < end0;
            const uint32_t g = in ? op_at(c, o).group : 0u;
            const bool first = in && (o == start || op_at(c, o - 1).group != g);
            const uint64_t mask = __ballot(first);
            const int idx = ng + __popcll(mask & ((1ull << tid) - 1ull));
            if (first && idx < kMaxPassGroups) {
                c.ug[idx].gidx = (int)g;
                c.ug[idx].a = o;
            }
            // the start of group kMaxPassGroups ends the pass
            const uint64_t over = __ballot(first && idx == kMaxPassGroups);
            ng += __popcll(mask);
            if (over) {
                end = __shfl(o, __ffsll((long long)over) - 1, 64);
                ng = kMaxPassGroups;
                break;
            }
        }
    }
    __syncthreads();
    // the lane's group record, written once every lane has read the ranges
    int rec_a = 0, rec_b = 0, rec_gidx = 0;
    uint32_t rec_flags = 0;
    if (tid < 64) {
        const int g = tid;
        int a = 0, b = 0, fb = 0, cu = 0, cm = 0;
        if (g < ng) {
            rec_gidx = c.ug[g].gidx;
            a = c.ug[g].a;
            b = g + 1 < ng ? c.ug[g + 1].a : end;
            fb = P.groups[rec_gidx].fallback ? 1 : 0;
            if (!fb) {
                group_shape(c, a, b, 1 << 30, 1 << 30, cu, cm);
                cu += 1;  // room for an even-count pad
            }
        }
        // exclusive scans over the groups
        int pu = cu, pm = cm;
#pragma unroll
        for (int s = 1; s < 64; s <<= 1) {
            const int xu = __shfl_up(pu, s, 64), xm = __shfl_up(pm, s, 64);
            if (tid >= s) {
                pu += xu;
                pm += xm;
            }
        }
        pu -= cu;
        pm -= cm;
        const bool fits = g >= ng || (pu + cu <= kMaxPassUops && pm + cm <= kMats);
        const uint64_t bad = __ballot(!fits);
        bool cut = end != end0;
        if (bad) {
            // the first group that does not fit is cut where the room ends
            const int gs = __ffsll((long long)bad) - 1;
            int o = 0;
            if (g == gs) {
                o = group_shape(c, a, b, kMaxPassUops - pu, kMats - pm, cu, cm);
                cu += 1;
                b = o;
            }
            o = __shfl(o, gs, 64);
            const int a_gs = __shfl(a, gs, 64);
            ng = o > a_gs ? gs + 1 : gs;
            end = o;
            cut = true;
        }
        unsigned long long flops = 0;
        int count = 0;
        if (g < ng && fb) {
            for (int o = a; o < b; ++o) flops += op_flops(P, op_at(c, o), c.dec[o - start]);
            rec_a = a;
            rec_b = b;
            rec_flags = kGrpFallback;
        } else if (g < ng) {
            const int ul = pu + cu, ml = pm + cm;
            int nu = pu, nm = pm;
            uint64_t fl = 0;
            PendRegs pr;
            pr.set = 0;
            for (int o = a; o < b; ++o) {
                const DevOp &op = op_at(c, o);
                const int d = c.dec[o - start];
                const double sc = (o == start && S.pending >= 0) ? S.first_scale : 1.0;
                if (op.kind == DK_BFUNC || ((op.flags & DF_COND) && d == kSkip)) continue;
                switch (op.kind) {
                case DK_MAT1:
                    fuse_factor(pr, op.rb[0], op_matrix_at(c, o, op), 1.0);
                    break;
                case DK_KRAUS: {
                    const DevRule &ru = rule_at(c, op.rule);
                    // c * I: the state is kept unnormalised anyway
                    if (((ru.scalar_mask >> d) & 1u) && sc == 1.0) break;
                    fuse_factor(pr, op.rb[0], P.pool + ru.mats + (size_t)d * 8, sc);
                    break;
                }
                case DK_PAULI: {
                    const uint32_t code = pauli_code_c(c, op.rule, rule_at(c, op.rule), d);
                    if (code == 0) break;  // identity
                    for (int t = 0; t < op.nq; ++t) {
                        const uint32_t x = (code >> t) & 1u, z = (code >> (8 + t)) & 1u;
                        if (!x && !z) continue;
                        // X = [[0,1],[1,0]], Z = [[1,0],[0,-1]], Y = [[0,-i],[i,0]]
                        double pmat[8] = {0, 0, 0, 0, 0, 0, 0, 0};
                        if (x && !z) { pmat[2] = 1; pmat[4] = 1; }
                        else if (!x && z) { pmat[0] = 1; pmat[6] = -1; }
                        else { pmat[3] = -1; pmat[5] = 1; }
                        fuse_factor(pr, op.rb[t], pmat, 1.0);
                    }
                    break;
                }
                default: {  // CX, CZ, SWAP
                    fuse_flush(c, pr, op.rb[0], nu, nm, ul, ml, fl, mf);
                    fuse_flush(c, pr, op.rb[1], nu, nm, ul, ml, fl, mf);
                    UOp u;
                    u.kind = op.kind == DK_CX ? UK_CX : op.kind == DK_CZ ? UK_CZ : UK_SWAP;
                    u.j0 = op.rb[0];
                    u.j1 = op.rb[1];
                    u.code = 0;
                    u.mat = 0;
                    u.pad2 = 0;
                    if (nu < ul) put_uop(c.uops + nu, u);
                    ++nu;
                }
                }
            }
            for (int jj = 0; jj < kMaxRegBits; ++jj) fuse_flush(c, pr, jj, nu, nm, ul, ml, fl, mf);
            if (nu + 1 > ul || nm > ml || (pr.set >> kMaxRegBits) != 0u) {
                // the counts disagree with what was built: run nothing, report it
                atomicOr(&P.ctl->error, kErrFuse);
                nu = pu;
            }
            rec_flags = pairs ? fold_trailing_perms(c.uops, pu, nu) : 0u;
            rec_a = pu;
            rec_b = nu - pu;
            count = nu - pu;
            flops = fl;
        }
        // totals over the groups
#pragma unroll
        for (int s = 32; s > 0; s >>= 1) {
            flops += __shfl_xor(flops, s, 64);
            count += __shfl_xor(count, s, 64);
        }
        if (tid == 0) {
            if (cut) {
                S.end = end;
                S.stop = STOP_NONE;
            }
            S.n_ug = ng;
            S.pass_flops = flops;
            S.st[ST_GROUPS] += ng;
            S.st[ST_UOPS] += count;
        }
    }
    __syncthreads();
    if (tid < ng) {
        c.ug[tid].gidx = rec_gidx;
        c.ug[tid].a = rec_a;
        c.ug[tid].b = rec_b;
        c.ug[tid].flags = rec_flags;
    }
    __syncthreads();
}

// ----------------------------------------------------------- reductions
// Squared norm and ||K_j v||^2 of a Kraus channel on NQ >= 2 tile bits
// b[0..NQ-1] (nm matrices of 2^NQ x 2^NQ FP64 complex at K), in FP64.
template <class R, int NQ>
__device__ void reduce_kraus_dense(Ctx<R> &c, const uint8_t *b, const double *K, int nm,
                                   double (&acc)[kMaxRed])
{
    constexpr int D = 1 << NQ;
    uint32_t bits[NQ], sorted[NQ];
#pragma unroll
    for (int t = 0; t < NQ; ++t) bits[t] = sorted[t] = b[t];
#pragma unroll
    for (int i = 0; i < NQ; ++i)
#pragma unroll
        for (int j = 0; j + 1 < NQ - i; ++j)
            if (sorted[j] > sorted[j + 1]) {
                const uint32_t t = sorted[j];
                sorted[j] = sorted[j + 1];
                sorted[j + 1] = t;
            }
    const uint32_t nbase = c.tsize >> NQ;
    for (uint32_t p = c.tid; p < nbase; p += kWG) {
        uint32_t base = p;
#pragma unroll
        for (int t = 0; t < NQ; ++t) base = ins0(base, sorted[t]);
        double vr[D], vi[D];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            uint32_t idx = base;
#pragma unroll
            for (int t = 0; t < NQ; ++t) idx |= ((uint32_t)(a >> t) & 1u) << bits[t];
            const auto v = c.L[c.at(idx)];
            vr[a] = v.x;
            vi[a] = v.y;
            acc[0] += fma(vr[a], vr[a], vi[a] * vi[a]);
        }
        for (int j = 0; j < nm && j < kMaxKraus; ++j) {
            const double *m = K + (size_t)j * D * D * 2;
            double sj = 0;
            for (int a = 0; a < D; ++a) {
                double wr = 0, wi = 0;
#pragma unroll
                for (int bb = 0; bb < D; ++bb) {
                    const double mr = m[2 * (a * D + bb)], mi = m[2 * (a * D + bb) + 1];
                    wr += mr * vr[bb] - mi * vi[bb];
                    wi += mr * vi[bb] + mi * vr[bb];
                }
                sj += fma(wr, wr, wi * wi);
            }
            acc[1 + j] += sj;
        }
    }
}

// Accumulate, over the tile, the squared norm and the candidate weights of
// op `op` (Kraus: ||K_j v||^2; measure: outcome probabilities).
template <class R>
__device__ __noinline__ void reduce_tile(Ctx<R> &c, const DevOp &op, double (&acc)[kMaxRed])
{
    using A = typename V2<R>::T;
    const ExecParams &P = c.P;
    lds<A> *L = c.L;
    if (op.kind == DK_KRAUS) {
        const DevRule &ru = P.rules[op.rule];
        const int nm = ru.n_terms;
        const double *K = P.pool + ru.mats;
        if (ru.nq == 1) {
            const uint32_t b = op.lb[0], half = c.tsize >> 1;
            for (uint32_t p = c.tid; p < half; p += kWG) {
                const uint32_t i0 = ins0(p, b), i1 = i0 | (1u << b);
                const A a = L[c.at(i0)], d = L[c.at(i1)];
                const double ar = a.x, ai = a.y, dr = d.x, di = d.y;
                acc[0] += fma(ar, ar, ai * ai) + fma(dr, dr, di * di);
#pragma unroll
                for (int j = 0; j < kMaxKraus; ++j) {
                    if (j >= nm) break;
                    const double *m = K + j * 8;
                    const double w0r = m[0] * ar - m[1] * ai + m[2] * dr - m[3] * di;
                    const double w0i = m[0] * ai + m[1] * ar + m[2] * di + m[3] * dr;
                    const double w1r = m[4] * ar - m[5] * ai + m[6] * dr - m[7] * di;
                    const double w1i = m[4] * ai + m[5] * ar + m[6] * di + m[7] * dr;
                    acc[1 + j] += fma(w0r, w0r, w0i * w0i) + fma(w1r, w1r, w1i * w1i);
                }
            }
        } else {
            switch (ru.nq) {
            case 2: reduce_kraus_dense<R, 2>(c, op.lb, K, nm, acc); break;
            case 3: reduce_kraus_dense<R, 3>(c, op.lb, K, nm, acc); break;
            case 4: reduce_kraus_dense<R, 4>(c, op.lb, K, nm, acc); break;
            default: reduce_kraus_dense<R, 5>(c, op.lb, K, nm, acc); break;
            }
        }
    } else {  // DK_MEASURE: only the op's 2^nq outcomes are accumulated
        const int no = 1 << op.nq;
        for (uint32_t i = c.tid; i < c.tsize; i += kWG) {
            uint32_t pat = 0;
            for (int t = 0; t < op.nq; ++t) pat |= ((i >> op.lb[t]) & 1u) << t;
            const double w = abs2d(L[c.at(i)]);
            acc[0] += w;
#pragma unroll
            for (int o = 0; o < 16; ++o) {
                if (o >= no) break;
                acc[1 + o] += (pat == (uint32_t)o) ? w : 0.0;
            }
        }
    }
}

// Sum acc[0..cnt) over the workgroup into S.red (fixed order).
template <class R>
__device__ __noinline__ void wg_reduce(Ctx<R> &c, double (&acc)[kMaxRed], int cnt)
{
    const int lane = c.tid & 63, wv = c.tid >> 6;
#pragma unroll
    for (int v = 0; v < kMaxRed; ++v) {
        if (v < cnt) {
            const double s = wave_sum(acc[v]);
            if (lane == 0) c.S.wred[v][wv] = s;
        }
    }
    __syncthreads();
    if (c.tid < cnt) {
        double s = 0;
        for (int w = 0; w < kWG / 64; ++w) s += c.S.wred[c.tid][w];
        c.S.red[c.tid] = s;
    }
    __syncthreads();
}

// Sum of one value over the workgroup; result valid in every thread.
template <class R>
__device__ double wg_sum1(Ctx<R> &c, double v)
{
    const int lane = c.tid & 63, wv = c.tid >> 6;
    const double s = wave_sum(v);
    if (lane == 0) c.S.wred[0][wv] = s;
    __syncthreads();
    double t = 0;
    for (int w = 0; w < kWG / 64; ++w) t += c.S.wred[0][w];
    __syncthreads();
    return t;
}

// ----------------------------------------------------------- tile I/O
template <class R>
__device__ __forceinline__ uint64_t tile_base(const PassInfo &pi, int n, int k, uint32_t t)
{
    uint64_t base = 0;
    for (int i = 0; i < n - k; ++i) base |= (uint64_t)((t >> i) & 1u) << pi.gq[i];
    return base;
}

__device__ __forceinline__ uint64_t tile_base_c(const cst<PassInfo> &pi, int n, int k, uint32_t t)
{
    // scalar loads are whole dwords: read the qubit bytes as words
    const cst<uint32_t> *w = (const cst<uint32_t> *)&pi + offsetof(PassInfo, gq) / 4;
    uint64_t base = 0;
    for (int i = 0; i < n - k; ++i)
        base |= (uint64_t)((t >> i) & 1u) << ((w[i >> 2] >> (8 * (i & 3))) & 0xffu);
    return base;
}

template <class R>
__device__ void build_hi_off(Ctx<R> &c, const PassInfo &pi, int k)
{
    const uint32_t nh = 1u << (k - kCoalesceQ);
    for (uint32_t h = c.tid; h < nh; h += kWG) {
        uint32_t off = 0;
        for (int i = 0; i < k - kCoalesceQ; ++i)
            off |= ((h >> i) & 1u) << pi.tq[kCoalesceQ + i];
        c.hi_off[h] = off;
    }
    __syncthreads();
}

// Global <-> LDS tile copies in 16-byte chunks (two c64 or one c128
// amplitude; the swizzle never touches bit 0, so a chunk stays contiguous),
// eight independent loads in flight per thread.
template <class R>
__device__ void load_tile(Ctx<R> &c, const gbl<typename V2<R>::T> *G, uint64_t base, bool fresh)
{
    using A = typename V2<R>::T;
    constexpr uint32_t V = 16 / sizeof(A);
    const uint32_t nch = c.tsize / V;
    if (fresh) {
        for (uint32_t ch = c.tid; ch < nch; ch += kWG) {
            const uint32_t l = ch * V;
            const uint64_t g = base + c.hi_off[l >> kCoalesceQ] + (l & kRunMask);
#pragma unroll
            for (uint32_t v = 0; v < V; ++v) {
                A z;
                z.x = (g + v == 0) ? (R)1 : (R)0;
                z.y = 0;
                c.L[c.at(l + v)] = z;
            }
        }
    } else if (nch % (8 * kWG) == 0) {
        for (uint32_t ch0 = c.tid; ch0 < nch; ch0 += 8 * kWG) {
            u32x4 x[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const uint32_t l = (ch0 + u * kWG) * V;
                x[u] = *(const gbl<u32x4> *)(G + base + c.hi_off[l >> kCoalesceQ] + (l & kRunMask));
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const uint32_t l = (ch0 + u * kWG) * V;
                *(lds<u32x4> *)(c.L + c.at(l)) = x[u];
            }
        }
    } else {
        for (uint32_t ch = c.tid; ch < nch; ch += kWG) {
            const uint32_t l = ch * V;
            *(lds<u32x4> *)(c.L + c.at(l)) = *(const gbl<u32x4> *)(G + base + c.hi_off[l >> kCoalesceQ] + (l & kRunMask));
        }
    }
    __syncthreads();
}

template <class R>
__device__ void store_tile(Ctx<R> &c, gbl<typename V2<R>::T> *G, uint64_t base)
{
    using A = typename V2<R>::T;
    constexpr uint32_t V = 16 / sizeof(A);
    for (uint32_t ch = c.tid; ch < c.tsize / V; ch += kWG) {
        const uint32_t l = ch * V;
        const uint64_t g = base + c.hi_off[l >> kCoalesceQ] + (l & kRunMask);
        *(gbl<u32x4> *)(G + g) = *(const lds<u32x4> *)(c.L + c.at(l));
    }
    __syncthreads();
}

template <class R>
__device__ __forceinline__ gbl<typename V2<R>::T> *slot_ptr(const ExecParams &P, int slot)
{
    using A = typename V2<R>::T;
    return (gbl<A> *)P.slots + (size_t)slot * P.slot_amps;
}

// ----------------------------------------------------------- queue/slots
__device__ bool spin_expired(unsigned long long t0, unsigned long long limit)
{
    return wall_clock64() - t0 > limit;
}

// Thread 0 only.
__device__ __noinline__ int slot_pop(const ExecParams &P)
{
    Control *ctl = P.ctl;
    const unsigned long long t0 = wall_clock64();
    while (atomicCAS(&ctl->lock, 0u, 1u) != 0u) {
        __builtin_amdgcn_s_sleep(2);
        if (spin_expired(t0, P.spin_limit)) {
            atomicOr(&ctl->error, kErrLock);
            return -1;
        }
    }
    __atomic_thread_fence(__ATOMIC_ACQUIRE);
    int s = -1;
    const int top = __hip_atomic_load(&ctl->free_top, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (top > 0) {
        s = __hip_atomic_load(&P.free_slots[top - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&ctl->free_top, top - 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __hip_atomic_store(&ctl->lock, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    return s;
}

__device__ __noinline__ void slot_push(const ExecParams &P, int s)
{
    Control *ctl = P.ctl;
    const unsigned long long t0 = wall_clock64();
    while (atomicCAS(&ctl->lock, 0u, 1u) != 0u) {
        __builtin_amdgcn_s_sleep(2);
        if (spin_expired(t0, P.spin_limit)) {
            atomicOr(&ctl->error, kErrLock);
            return;
        }
    }
    __atomic_thread_fence(__ATOMIC_ACQUIRE);
    const int top = __hip_atomic_load(&ctl->free_top, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (top < P.n_slots) {
        __hip_atomic_store(&P.free_slots[top], s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&ctl->free_top, top + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
        atomicOr(&ctl->error, kErrState);
    }
    __hip_atomic_store(&ctl->lock, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Thread 0 only: reserve a record, fill it, publish it.
__device__ __noinline__ void queue_push(const ExecParams &P, const BranchRec &r)
{
    Control *ctl = P.ctl;
    const uint32_t idx = atomicAdd(&ctl->q_tail, 1u);
    if (idx >= (uint32_t)P.queue_cap) {
        atomicOr(&ctl->error, kErrQueue);
        return;
    }
    atomicAdd(&ctl->outstanding, 1);
    P.queue[idx] = r;
    __threadfence();
    st_rel(&P.ready[idx], 1u);
}

// ----------------------------------------------------------- decisions
__device__ __forceinline__ int pauli_pick(const ExecParams &P, const DevRule &ru, double u)
{
    const double *thr = P.pool + ru.thr;
    for (int j = 0; j < (int)ru.n_terms; ++j)
        if (u < thr[j]) return j;
    return (int)ru.n_terms - 1;
}

// Relative decision margin: distance from x to the running-sum boundaries
// that separate the chosen candidate j from its neighbours (prev = C_{j-1}
// if j > 0, cur = C_j if j is not the last candidate), over N. A choice made
// by the rounding fall-back has margin 0.
__device__ __forceinline__ double rel_margin(double x, double N, int j, int cnt, double prev,
                                             double cur, bool fell_back)
{
    if (fell_back || !(N > 0)) return 0.0;
    double m = __builtin_inf();
    if (j > 0) m = fmin(m, x - prev);
    if (j < cnt - 1) m = fmin(m, cur - x);
    return m / N;
}

// First candidate whose running sum of S.red[1..] exceeds u*N; if rounding
// leaves none, the last candidate with a non-zero weight. N is the squared
// norm of the same sweep: for a Kraus channel its own sum (S.red[0]), for a
// measurement the sum of the outcome probabilities in outcome order.
__device__ __forceinline__ int red_pick(const lds<WgShared> &S, int cnt, double u,
                                        bool norm_from_outcomes, double &margin)
{
    double N = S.red[0];
    if (norm_from_outcomes) {
        N = 0;
        for (int o = 0; o < cnt; ++o) N += S.red[1 + o];
    }
    const double x = u * N;
    double run = 0, prev = 0;
    int last = -1;
    for (int o = 0; o < cnt; ++o) {
        const double p = S.red[1 + o];
        if (p > 0) last = o;
        prev = run;
        run += p;
        if (x < run) {
            margin = rel_margin(x, N, o, cnt, prev, run, false);
            return o;
        }
    }
    margin = 0.0;
    return last < 0 ? 0 : last;
}

__device__ __forceinline__ int red_count(const ExecParams &P, const DevOp &op)
{
    return op.kind == DK_KRAUS ? (int)P.rules[op.rule].n_terms : (1 << op.nq);
}

// Record measured bits (with readout flips) of shot `shot`.
// A shot's classical register is read back on the device (conditions,
// branch ops) after other waves wrote it: device-scope accesses, which do
// not stop at a compute unit's own cache.
__device__ __forceinline__ uint64_t creg_load(const uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void creg_store(uint64_t *p, uint64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __noinline__ void record_bits(const ExecParams &P, const DevOp &op, uint64_t shot, uint32_t o)
{
    uint64_t m = creg_load(P.memory + shot);
    for (int t = 0; t < op.nq; ++t) {
        uint64_t bit = (o >> t) & 1u;
        const double pf = bit ? P.ro10 : P.ro01;
        if (pf > 0 && philox_u01(P.seed, P.shot_base + shot, op.r, 1u + t) < pf) bit ^= 1u;
        m = (m & ~(1ull << op.c[t])) | (bit << op.c[t]);
    }
    creg_store(P.memory + shot, m);
}

// Outcome of shot `shot` at random op `op` (after its reduction, if any),
// with the relative margin of a state-dependent choice (+inf for a Pauli
// draw, whose thresholds are host constants).
__device__ __forceinline__ int outcome_of(const ExecParams &P, const lds<WgShared> &S,
                                          const DevOp &op, uint64_t shot, double &margin)
{
    const double u = philox_u01(P.seed, P.shot_base + shot, op.r, 0);
    margin = __builtin_inf();
    if (op.kind == DK_PAULI) return pauli_pick(P, P.rules[op.rule], u);
    return red_pick(S, red_count(P, op), u, op.kind == DK_MEASURE, margin);
}

// Keep the smallest decision margin of a shot (device-scope accesses: the
// shot's record may have been run by other workgroups before). Returns 1
// for a near-tie.
__device__ __forceinline__ int note_margin(const ExecParams &P, uint64_t shot, double m)
{
    if (!(m < __builtin_inf())) return 0;
    const uint64_t bits = __builtin_bit_cast(uint64_t, m);
    if (bits < creg_load(P.margins + shot)) creg_store(P.margins + shot, bits);
    return m < kNearTie ? 1 : 0;
}

// Value of a condition (or branch-op predicate) for one shot.
__device__ __forceinline__ int cond_of(const ExecParams &P, const DevOp &op, uint64_t shot)
{
    return (creg_load(P.memory + shot) & op.cond_mask) == op.cond_value ? 1 : 0;
}

// Classical-register op of the record's shots (Sec. IV-A): a branch op
// writes each shot's clbit; a condition is evaluated for every shot.
// Returns 0 (false for every shot), 1 (true for every shot) or 2 (mixed).
template <class R>
__device__ __noinline__ int creg_op(Ctx<R> &c, const DevOp &op)
{
    const ExecParams &P = c.P;
    lds<WgShared> &S = c.S;
    if (c.tid == 0) { S.omin = 1; S.omax = 0; }
    __syncthreads();
    int lmin = 1, lmax = 0;
    for (int i = S.lo + c.tid; i < S.hi; i += kWG) {
        const uint64_t shot = (uint64_t)P.shot_perm[i];
        const uint64_t creg = creg_load(P.memory + shot);
        const int t = (creg & op.cond_mask) == op.cond_value ? 1 : 0;
        if (op.kind == DK_BFUNC)
            creg_store(P.memory + shot, (creg & ~(1ull << op.c[0])) | ((uint64_t)t << op.c[0]));
        lmin = min(lmin, t);
        lmax = max(lmax, t);
    }
    if (lmin == 0) atomicMin((int *)&S.omin, 0);
    if (lmax == 1) atomicMax((int *)&S.omax, 1);
    __syncthreads();  // also orders the branch op's stores before later reads
    const int r = S.omin == S.omax ? S.omin : 2;
    __syncthreads();
    return r;
}

// ----------------------------------------------------------- the kernel
template <class R>
__device__ __noinline__ void copy_state_to_slot(Ctx<R> &c, int dst, int src_slot, bool from_lds)
{
    using A = typename V2<R>::T;
    const ExecParams &P = c.P;
    gbl<A> *D = slot_ptr<R>(P, dst);
    const uint64_t namps = 1ull << P.n_qubits;
    if (from_lds) {
        for (uint64_t i = c.tid; i < namps; i += kWG) D[i] = c.L[i];
    } else {
        const gbl<u32x4> *Sp = (const gbl<u32x4> *)slot_ptr<R>(P, src_slot);
        gbl<u32x4> *Dp = (gbl<u32x4> *)D;
        const uint64_t n16 = namps * sizeof(A) / 16;
        for (uint64_t i = c.tid; i < n16; i += kWG) Dp[i] = Sp[i];
    }
    __threadfence();
    __syncthreads();
}

// Partition the branch's shots by outcome at op j and continue with the
// first group; other groups get a copied state (or the waiting list).
template <class R>
__device__ __noinline__ void split_branch(Ctx<R> &c, const DevOp &op, int j, bool cnd)
{
    const ExecParams &P = c.P;
    lds<WgShared> &S = c.S;
    const int tid = c.tid;
    // cnd: the op's condition differs between the record's shots, which are
    // split by its value; each part then finds it uniform and runs or skips
    // the op. Otherwise the split is by the op's drawn outcome.
    const int m = S.hi - S.lo;
    const int chunk = (m + kWG - 1) / kWG;
    const int my_lo = S.lo + min(m, tid * chunk), my_hi = S.lo + min(m, (tid + 1) * chunk);
    // Shots are grouped into 16 buckets. The bucket of an outcome is the
    // outcome itself, except for a Pauli channel of more than 16 terms:
    // there it is the rank of the drawn term among the terms drawn in this
    // record, and when more than 16 distinct terms are drawn, ranks from
    // 15 on share bucket 15, whose shots are left undecided and split
    // again by their own record (at least 15 terms are settled per split)
    // (bitmap of the drawn terms and its prefix counts in the pass's
    // decision area, unused between the sweep and the next plan)
    const bool ranked = !cnd && op.kind == DK_PAULI && P.rules[op.rule].n_terms > 16;
    constexpr int kW = kMaxPauliTerms / 32;
    static_assert(2 * kW * 4 <= kMaxPassOps * 2, "term bitmap fits the decision area");
    lds<uint32_t> *obits = (lds<uint32_t> *)c.dec;
    lds<int> *obase = (lds<int> *)(obits + kW);
    if (ranked) {
        for (int w = tid; w < kW; w += kWG) obits[w] = 0;
        __syncthreads();
        for (int i = my_lo; i < my_hi; ++i) {
            double mg;
            const int o = outcome_of(P, S, op, (uint64_t)P.shot_perm[i], mg);
            atomicOr((uint32_t *)&obits[o >> 5], 1u << (o & 31));
        }
        __syncthreads();
        if (tid == 0) {
            int run = 0;
            for (int w = 0; w < kW; ++w) {
                obase[w] = run;
                run += __popc(obits[w]);
            }
            S.n_distinct = run;
        }
        __syncthreads();
    }
    auto bucket_of = [&](int o) -> int {
        if (!ranked) return o;
        const int r = obase[o >> 5] + __popc(obits[o >> 5] & ((1u << (o & 31)) - 1u));
        return r < 15 ? r : 15;
    };
    int my_cnt[16];
#pragma unroll
    for (int o = 0; o < 16; ++o) my_cnt[o] = 0;
    for (int i = my_lo; i < my_hi; ++i) {
        const uint64_t sh = (uint64_t)P.shot_perm[i];
        double mg;
        const int o = bucket_of(cnd ? cond_of(P, op, sh) : outcome_of(P, S, op, sh, mg));
#pragma unroll
        for (int q = 0; q < 16; ++q) my_cnt[q] += (o == q);
    }
#pragma unroll
    for (int o = 0; o < 16; ++o) c.cnt[o * kWG + tid] = my_cnt[o];
    __syncthreads();
    if (tid < 16) {  // exclusive scan of row `tid` over threads
        int run = 0;
        for (int t = 0; t < kWG; ++t) {
            const int v = c.cnt[tid * kWG + t];
            c.cnt[tid * kWG + t] = run;
            run += v;
        }
        S.tot[tid] = run;
    }
    __syncthreads();
    if (tid == 0) {
        int off = S.lo, g = 0;
        for (int o = 0; o < 16; ++o) {
            if (S.tot[o] == 0) continue;
            int val = o;  // the outcome of bucket o (-1: undecided)
            if (ranked) {
                val = -1;
                if (o < 15 || S.n_distinct <= 16) {
                    int seen = 0;
                    for (int w = 0; w < kW && val < 0; ++w) {
                        const uint32_t bw = obits[w];
                        if (seen + __popc(bw) > o) {
                            uint32_t x = bw;
                            for (int k = seen; k < o; ++k) x &= x - 1u;  // drop lower set bits
                            val = w * 32 + __builtin_ctz(x);
                        }
                        seen += __popc(bw);
                    }
                }
            }
            S.grp_o[g] = val;
            S.grp_lo[g] = off;
            S.grp_hi[g] = off + S.tot[o];
            off += S.tot[o];
            ++g;
        }
        S.n_groups = g;
        // a condition split must divide the record, else it would recur
        // forever at the same op: end the record with an error instead
        if (cnd && g < 2) {
            atomicOr(&P.ctl->error, kErrState);
            S.n_groups = 0;
        }
    }
    __syncthreads();
    if (S.n_groups == 0) {
        if (tid == 0) {
            S.cursor = P.n_ops;
            S.pending = -1;
        }
        __syncthreads();
        return;
    }
    // scatter into shot_tmp, then copy back
    {
        // groups are in bucket order: group g holds the g-th non-empty bucket
        int pos[16];
        {
            int g = 0;
            for (int o = 0; o < 16; ++o) {
                const int base = S.tot[o] ? S.grp_lo[g++] : 0;
                pos[o] = base + c.cnt[o * kWG + tid];
            }
        }
        int ties = 0;
        for (int i = my_lo; i < my_hi; ++i) {
            const int shot = P.shot_perm[i];
            double mg = __builtin_inf();
            const int o = cnd ? cond_of(P, op, (uint64_t)shot) : outcome_of(P, S, op, (uint64_t)shot, mg);
            if (!cnd) ties += note_margin(P, (uint64_t)shot, mg);
            const int bk = bucket_of(o);
            int p = 0;
#pragma unroll
            for (int q = 0; q < 16; ++q)
                if (bk == q) p = pos[q]++;
            P.shot_tmp[p] = shot;
            if (!cnd && op.kind == DK_MEASURE && (op.flags & DF_RECORD))
                record_bits(P, op, (uint64_t)shot, (uint32_t)o);
        }
        if (ties) atomicAdd((unsigned long long *)&S.st[ST_NEARTIES], (unsigned long long)ties);
    }
    __threadfence_block();
    __syncthreads();
    for (int i = S.lo + tid; i < S.hi; i += kWG) P.shot_perm[i] = P.shot_tmp[i];
    __syncthreads();

    const bool measure_like = op.kind != DK_PAULI && !cnd;
    for (int g = 1; g < S.n_groups; ++g) {
        const int o = S.grp_o[g];
        const double sc = measure_like ? 1.0 / sqrt(S.red[1 + o]) : 1.0;
        if (tid == 0) S.alloc_slot = slot_pop(P);
        __syncthreads();
        const int slot = S.alloc_slot;
        // a parent that was never written is still |0..0>: no copy needed
        const bool child_fresh = S.fresh && !P.resident;
        if (slot >= 0) {
            if (!child_fresh) copy_state_to_slot(c, slot, S.slot, P.resident != 0);
            if (tid == 0) {
                BranchRec r;
                r.slot = slot;
                r.lo = S.grp_lo[g];
                r.hi = S.grp_hi[g];
                r.cursor = j;
                r.pending = cnd ? -1 : o;
                r.flags = child_fresh ? 1 : 0;
                r.scale = sc;
                r.norm_lb = measure_like ? 1.0 : S.norm_lb;
                S.st[ST_BRANCHES] += 1;
                queue_push(P, r);
            }
        } else {
            const int cntg = S.grp_hi[g] - S.grp_lo[g];
            if (tid == 0) {
                S.wait_base = (int)atomicAdd(&P.ctl->wait_count, (uint32_t)cntg);
                S.st[ST_WAITING] += cntg;
            }
            __syncthreads();
            for (int i = tid; i < cntg; i += kWG) P.waiting[S.wait_base + i] = P.shot_perm[S.grp_lo[g] + i];
        }
        __syncthreads();
    }
    if (tid == 0) {
        const int o = S.grp_o[0];
        S.lo = S.grp_lo[0];
        S.hi = S.grp_hi[0];
        S.cursor = j;
        S.pending = cnd ? -1 : o;
        S.first_scale = measure_like ? 1.0 / sqrt(S.red[1 + o]) : 1.0;
        if (measure_like) S.norm_lb = 1.0;
        S.st[ST_SPLITS] += 1;
    }
    __syncthreads();
}

// Determine the op range of the next sweep (and why it stops).
// All threads: copy op records [first, first + cnt) of the program, and the
// matrices of their DK_MAT1 ops, to the LDS staging area, so that the
// pass's planning and fusion (one thread, op after op) read LDS, not global
// memory. Ends with a barrier.
template <class R>
__device__ __noinline__ void stage_ops(Ctx<R> &c, int first, int cnt)
{
    const ExecParams &P = c.P;
    constexpr int W = (int)(sizeof(DevOp) / 16);
    const gbl<u32x4> *src = (const gbl<u32x4> *)(P.ops + first);
    lds<u32x4> *dst = (lds<u32x4> *)(lds<DevOp> *)c.sops;
    for (int i = c.tid; i < cnt * W; i += kWG) dst[i] = src[i];
    for (int i = c.tid; i < cnt; i += kWG) {
        const DevOp &op = P.ops[first + i];
        if (op.kind != DK_MAT1) continue;
        const double *m = op_matrix(P, op, c.S);
#pragma unroll
        for (int e = 0; e < 8; ++e) c.smat[i * 8 + e] = m[e];
    }
    c.s0 = first;
    c.scap = cnt;
    __syncthreads();
}

template <class R>
__device__ __noinline__ void plan_pass(Ctx<R> &c)
{
    const ExecParams &P = c.P;
    lds<WgShared> &S = c.S;
    const int tid = c.tid;
    const int start = S.cursor;
    const int m = S.hi - S.lo;
    int j = start;
    if (start >= P.n_ops) {
        if (tid == 0) { S.start = S.end = start; S.stop = STOP_END; }
        __syncthreads();
        return;
    }
    const PassInfo &pi = P.passes[P.ops[start].pass];
    const int end_static = (int)pi.end_op;
    int lim = kMaxPassOps;  // ops in this pass at most
    if (P.stage_cap > 0) {
        lim = min(P.stage_cap, end_static - start);
        stage_ops(c, start, lim);
    }
    if (S.pending >= 0) {
        if (tid == 0) c.dec[0] = S.pending;
        ++j;
    }
    if (m == 1) {
        // one shot: its Pauli draws depend neither on each other nor on the
        // state, so every op of the window is drawn at once, one per thread
        // (a draw past where the pass stops is drawn again by the next pass)
        const uint64_t shot = (uint64_t)P.shot_perm[S.lo];
        const int jend = min(end_static, start + lim);
        for (int q = j + tid; q < jend; q += kWG) {
            const DevOp &o = op_at(c, q);
            if (o.kind != DK_PAULI) continue;
            const double u = philox_u01(P.seed, P.shot_base + shot, o.r, 0);
            c.dec[q - start] = (int16_t)pauli_pick_c(c, o.rule, rule_at(c, o.rule), u);
        }
        __syncthreads();
    }
    double nlb = S.norm_lb;
    int stop = STOP_NONE;
    const double lb_floor = sizeof(R) == 4 ? 0x1.0p-30 : 0x1.0p-200;
    for (;;) {
        while (j < end_static && j - start < lim) {
            const DevOp &oj = op_at(c, j);
            const uint16_t kd = oj.kind;
            if ((kd == DK_PAULI && m != 1) || kd == DK_KRAUS || kd == DK_MEASURE ||
                kd == DK_BFUNC || (oj.flags & DF_COND))
                break;
            ++j;
        }
        if (j >= end_static || j - start >= lim) break;
        const DevOp &op = op_at(c, j);
        if (op.kind == DK_BFUNC || (op.flags & DF_COND)) {
            const int v = creg_op(c, op);
            if (op.kind == DK_BFUNC || v == 0) {  // done / skipped for every shot
                if (tid == 0) c.dec[j - start] = kSkip;
                ++j;
                continue;
            }
            if (v == 2) {
                if (tid == 0) S.split_cond = 1;
                stop = STOP_SPLIT;
                break;
            }
            if (op.kind != DK_PAULI && op.kind != DK_KRAUS && op.kind != DK_MEASURE) {
                if (tid == 0) c.dec[j - start] = 0;  // a gate whose condition holds for every shot
                ++j;
                continue;
            }
        }
        if (op.kind == DK_MEASURE) {
            stop = (op.flags & DF_TERMINAL) ? STOP_TERMINAL : STOP_REDUCE;
            break;
        }
        const DevRule &ru = rule_at(c, op.rule);
        if (m == 1) {
            if (op.kind == DK_PAULI) {  // drawn above
                ++j;
                continue;
            }
            // every thread evaluates the single shot's draw (no barrier)
            const uint64_t shot = (uint64_t)P.shot_perm[S.lo];
            const double u = philox_u01(P.seed, P.shot_base + shot, op.r, 0);
            if (u < ru.lam_min0 && nlb * ru.lam_min0 >= lb_floor) {
                if (tid == 0) c.dec[j - start] = 0;
                if (!(ru.scalar_mask & 1u)) nlb *= ru.lam_min0;
                ++j;
                continue;
            }
            stop = STOP_REDUCE;
            break;
        }
        // several shots: evaluate all draws, agree on the outcome
        if (tid == 0) { S.omin = 1 << 30; S.omax = -1; S.anyhigh = 0; }
        __syncthreads();
        int lmin = 1 << 30, lmax = -1, high = 0;
        for (int i = S.lo + tid; i < S.hi; i += kWG) {
            const uint64_t shot = (uint64_t)P.shot_perm[i];
            const double u = philox_u01(P.seed, P.shot_base + shot, op.r, 0);
            if (op.kind == DK_PAULI) {
                const int o = pauli_pick_c(c, op.rule, ru, u);
                lmin = min(lmin, o);
                lmax = max(lmax, o);
            } else if (!(u < ru.lam_min0)) {
                high = 1;
            }
        }
        if (op.kind == DK_PAULI) {
            atomicMin((int *)&S.omin, lmin);
            atomicMax((int *)&S.omax, lmax);
        } else if (high) {
            atomicOr((int *)&S.anyhigh, 1);
        }
        __syncthreads();
        const int omin = S.omin, omax = S.omax, anyhigh = S.anyhigh;
        __syncthreads();
        if (op.kind == DK_PAULI) {
            if (omin == omax) {
                if (tid == 0) c.dec[j - start] = omin;
                ++j;
                continue;
            }
            if (tid == 0) S.split_cond = 0;
            stop = STOP_SPLIT;
            break;
        }
        if (!anyhigh && nlb * ru.lam_min0 >= lb_floor) {
            if (tid == 0) c.dec[j - start] = 0;
            if (!(ru.scalar_mask & 1u)) nlb *= ru.lam_min0;
            ++j;
            continue;
        }
        stop = STOP_REDUCE;
        break;
    }
    if (tid == 0) {
        S.start = start;
        S.end = j;
        S.stop = stop;
        S.stop_op = j;
        S.norm_lb = nlb;
        S.n_ug = 0;
        S.pass_flops = 0;
    }
    __syncthreads();
    if (P.use_groups && j > start) build_uops(c);  // ends with a barrier
}

template <class R>
__device__ void apply_range(Ctx<R> &c, uint64_t &flops)
{
    const ExecParams &P = c.P;
    lds<WgShared> &S = c.S;
    for (int j = S.start; j < S.end; ++j) {
        const DevOp &op = op_at(c, j);
        const int d = c.dec[j - S.start];
        const double s = (j == S.start && S.pending >= 0) ? S.first_scale : 1.0;
        apply_op(c, op, d, s);
        flops += op_flops(P, op, d);
    }
}

// A fallback group: its ops run as LDS sweeps over the current tile.
template <class R>
__device__ __noinline__ void run_fallback(Ctx<R> &c, int a, int b)
{
    lds<WgShared> &S = c.S;
    for (int o = a; o < b; ++o) {
        const double s = (o == S.start && S.pending >= 0) ? S.first_scale : 1.0;
        apply_op(c, op_at(c, o), c.dec[o - S.start], s);
    }
}

// The pass's groups on the current tile, in order. With d, a last group
// that runs in registers stores the tile to HBM itself (returns true).
template <class R, int NR, bool MF>
__device__ __forceinline__ bool run_groups(Ctx<R> &c, const Hot &h, const cst<GroupInfo> *groups,
                                           bool direct, const Direct<R, NR> &d)
{
    bool stored = false;
    for (int u = 0; u < h.n_ug; ++u) {
        const lds<UGroup> &gl = ((const lds<UGroup> *)(size_t)h.ug)[u];
        const int gidx = (int)uni((uint32_t)gl.gidx);
        const int a = (int)uni((uint32_t)gl.a);
        const int b = (int)uni((uint32_t)gl.b);
        const uint32_t gfl = uni(gl.flags);
        const int fb = (int)(gfl & kGrpFallback);
        if (fb) {
            run_fallback<R>(c, a, b);
        } else if constexpr (NR > 0) {
            const bool last_direct = direct && u == h.n_ug - 1;
            run_group<R, NR, MF>(h, groups[gidx], a, b, gfl, last_direct, d);
            stored = stored || last_direct;
        }
    }
    return stored;
}

template <class R, int NR, bool MF>
__device__ void run_sweep(Ctx<R> &c, bool want_reduce)
{
    using A = typename V2<R>::T;
    const ExecParams &P = c.P;
    lds<WgShared> &S = c.S;
    const int n = P.n_qubits, k = P.tile_q;
    const bool has_ops = S.end > S.start;
    const bool grp = NR > 0 && P.use_groups && !P.resident && has_ops;
    double acc[kMaxRed];
#pragma unroll
    for (int v = 0; v < kMaxRed; ++v) acc[v] = 0;
    const DevOp &rop = P.ops[S.stop_op < P.n_ops ? S.stop_op : 0];
    uint64_t flops = 0;
    if (P.resident) {
        bool done = false;
        if constexpr (NR > 0) {
            // the whole state sits in LDS (unswizzled): register groups
            // gather from it and scatter back, with no HBM traffic
            if (P.use_groups && has_ops) {
                Hot h;
                h.ug = (uint32_t)(size_t)c.ug;
                h.uops = (uint32_t)(size_t)c.uops;
                h.mats = (uint32_t)(size_t)c.mats;
                h.lbase = 0;
                h.hi = (uint32_t)(size_t)c.hi_off;
                h.swm = 0;
                h.n_ug = (int)uni((uint32_t)S.n_ug);
                h.k = k;
                h.tid = c.tid;
                TileIO<R, NR> io{};  // no tile copies
                run_groups<R, NR, MF>(c, h, to_const(P.groups), false,
                                  Direct<R, NR>{nullptr, nullptr, 0, false, io});
                flops = S.pass_flops;
                done = true;
            }
        }
        if (!done) apply_range(c, flops);
        if (want_reduce) reduce_tile(c, rop, acc);
    } else {
        const PassInfo &pi = P.passes[P.ops[S.start].pass];
        c.swm = P.use_groups ? P.swz : 0u;
        build_hi_off(c, pi, k);
        gbl<A> *G = slot_ptr<R>(P, S.slot);
        const bool fresh = S.fresh != 0;
        if constexpr (NR > 0) {
            if (P.use_groups) {
                Hot h;
                h.ug = (uint32_t)(size_t)c.ug;
                h.uops = (uint32_t)(size_t)c.uops;
                h.mats = (uint32_t)(size_t)c.mats;
                h.lbase = 0;
                h.hi = (uint32_t)(size_t)c.hi_off;
                h.swm = uni(c.swm);
                h.n_ug = (int)uni((uint32_t)S.n_ug);
                h.k = k;
                h.tid = c.tid;
                const cst<GroupInfo> *groups = to_const(P.groups);
                const cst<PassInfo> &pc = *to_const(&pi);
                TileIO<R, NR> io;
                io.setup_linear(c);
                // nothing below may read private memory: such a load would
                // wait for the tile copy in flight
                const uint32_t nt = uni(1u << (n - k));
                if (P.nbuf == 2 && !fresh) {
                    const uint32_t tb = uni((1u << k) * (uint32_t)sizeof(A));  // buffer 1 starts here
                    lds<A> *const L0 = c.L;
                    io.issue(G, tile_base_c(pc, n, k, 0), 0);
                    for (uint32_t t = 0; t < nt; ++t) {
                        const uint32_t cur = (t & 1u) ? tb : 0u;
                        wait_vm();
                        __syncthreads();
                        if (t + 1 < nt) io.issue(G, tile_base_c(pc, n, k, t + 1), cur ^ tb);
                        h.lbase = cur;
                        c.lbase = cur;  // cold paths (fallback groups, reductions) use c.L
                        c.L = (lds<A> *)((lds<unsigned char> *)L0 + cur);
                        if (grp) run_groups<R, NR, MF>(c, h, groups, false, Direct<R, NR>{G, G, 0, false, io});
                        if (want_reduce) reduce_tile(c, rop, acc);
                        if (has_ops) io.store_linear(G, tile_base_c(pc, n, k, t), cur);
                    }
                    c.lbase = 0;
                    c.L = L0;
                } else {
                    // one buffer, filled by asynchronous global->LDS copies
                    // (no register staging) and drained in linear order, or
                    // by the last register group straight from registers
                    const bool direct = grp && !want_reduce;
                    if (!fresh) io.issue(G, tile_base_c(pc, n, k, 0), 0);
                    for (uint32_t t = 0; t < nt; ++t) {
                        const uint64_t base = tile_base_c(pc, n, k, t);
                        const bool more = !fresh && t + 1 < nt;
                        const uint64_t next = more ? tile_base_c(pc, n, k, t + 1) : 0;
                        if (fresh) io.zero(base == 0);
                        wait_vm();
                        __syncthreads();
                        bool stored = false;
                        if (grp) {
                            stored = run_groups<R, NR, MF>(c, h, groups, direct,
                                                       Direct<R, NR>{G + base, G, next, more, io});
                        }
                        if (want_reduce) reduce_tile(c, rop, acc);
                        if (!stored) {
                            if (has_ops) io.store_linear(G, base, 0);
                            lds_sync();  // the buffer is read out before the next copy lands
                            if (more) io.issue(G, next, 0);
                        }
                    }
                }
                wait_vm();  // the next pass reads what these stores write
                __syncthreads();
            }
        }
        if (!(NR > 0 && P.use_groups)) {
            for (uint32_t t = 0; t < c.n_tiles; ++t) {
                const uint64_t base = tile_base<R>(pi, n, k, t);
                load_tile(c, G, base, fresh);
                apply_range(c, flops);
                if (want_reduce) {
                    reduce_tile(c, rop, acc);
                }
                if (has_ops) store_tile(c, G, base);
            }
        }
        c.swm = 0;
        if (grp) flops = S.pass_flops * c.n_tiles;
        if (c.tid == 0) {
            const uint64_t sb = (1ull << n) * sizeof(A);
            S.st[ST_PASSES] += 1;
            S.st[ST_BYTES] += (fresh ? 0 : sb) + (has_ops ? sb : 0);
        }
        if (has_ops) {
            __syncthreads();
            if (c.tid == 0) S.fresh = 0;
        }
    }
    if (c.tid == 0) {
        S.st[ST_FLOPS] += flops * (uint64_t)c.tsize;
        __hip_atomic_fetch_add(&P.ctl->heartbeat, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (want_reduce) {
        wg_reduce(c, acc, 1 + red_count(P, rop));
        if (c.tid == 0) S.st[ST_REDUCTIONS] += 1;
    }
    __syncthreads();
}

// After a reduction for op j: each shot's outcome; continue with it, or
// split the branch.
template <class R>
__device__ __noinline__ void decide(Ctx<R> &c)
{
    const ExecParams &P = c.P;
    lds<WgShared> &S = c.S;
    const int j = S.stop_op;
    const DevOp &op = P.ops[j];
    const int m = S.hi - S.lo;
    if (m == 1) {
        if (c.tid == 0) {
            const uint64_t shot = (uint64_t)P.shot_perm[S.lo];
            double mg;
            const int o = outcome_of(P, S, op, shot, mg);
            S.st[ST_NEARTIES] += note_margin(P, shot, mg);
            if (op.kind == DK_MEASURE && (op.flags & DF_RECORD)) record_bits(P, op, shot, (uint32_t)o);
            S.cursor = j;
            S.pending = o;
            S.first_scale = 1.0 / sqrt(S.red[1 + o]);
            S.norm_lb = 1.0;
        }
        __syncthreads();
        return;
    }
    if (P.branch_mode) {
        split_branch(c, op, j, false);  // by outcome, whatever split came before
        return;
    }
    // several shots on one state without splitting cannot happen
    if (c.tid == 0) {
        atomicOr(&P.ctl->error, kErrState);
        S.cursor = P.n_ops;
        S.pending = -1;
    }
    __syncthreads();
}

// Final measurement of all qubits by sampling the shared state once per
// shot: FP64 tile sums, tile search, in-tile prefix and search.
template <class R>
__device__ __noinline__ void terminal_sample(Ctx<R> &c)
{
    using A = typename V2<R>::T;
    const ExecParams &P = c.P;
    lds<WgShared> &S = c.S;
    const int n = P.n_qubits, k = P.tile_q;
    const int tid = c.tid;
    const DevOp &op = P.ops[S.stop_op];
    lds<double> *D = (lds<double> *)c.L;  // in-place |a|^2 prefix, same bytes as the tile
    double *tsums = P.tile_sums + (size_t)blockIdx.x * c.n_tiles;
    const PassInfo &pi = P.passes[op.pass];
    gbl<A> *G = P.resident ? nullptr : slot_ptr<R>(P, S.slot);
    const uint32_t seg = c.tsize >= kWG ? c.tsize / kWG : 1;

    // in-tile: D[e] = inclusive prefix of |a|^2 in the tile (LDS)
    auto tile_prefix = [&](void) {
        double vals[32];
        const uint32_t my0 = tid * seg;
        const bool active = my0 < c.tsize;
        double run = 0;
        if (sizeof(A) == 8) {
            if (active)
                for (uint32_t e = 0; e < seg; ++e) {
                    run += abs2d(c.L[my0 + e]);
                    D[my0 + e] = run;
                }
            __syncthreads();
        } else {
            // 16-byte amplitudes overlap other threads' doubles: read first
            for (uint32_t e0 = 0; e0 < seg; e0 += 32) {
                const uint32_t cntv = min(32u, seg - e0);
                if (active)
                    for (uint32_t e = 0; e < cntv; ++e) vals[e] = abs2d(c.L[my0 + e0 + e]);
                __syncthreads();
                if (active)
                    for (uint32_t e = 0; e < cntv; ++e) {
                        run += vals[e];
                        D[my0 + e0 + e] = run;
                    }
                __syncthreads();
            }
        }
        // segment offsets (sequential over segments, fixed order)
        lds<double> *off = (lds<double> *)c.scr;   // kWG doubles
        if (active) off[tid] = run; else if (tid < kWG) off[tid] = 0;
        __syncthreads();
        if (tid == 0) {
            double r2 = 0;
            for (int t = 0; t < kWG; ++t) {
                const double v = off[t];
                off[t] = r2;
                r2 += v;
            }
        }
        __syncthreads();
        if (active) {
            const double o = off[tid];
            for (uint32_t e = 0; e < seg; ++e) D[my0 + e] += o;
        }
        __syncthreads();
    };

    if (P.resident) {
        tile_prefix();
        if (tid == 0) { tsums[0] = D[c.tsize - 1]; }
        __syncthreads();
    } else {
        build_hi_off(c, pi, k);
        for (uint32_t t = 0; t < c.n_tiles; ++t) {
            const uint64_t base = tile_base<R>(pi, n, k, t);
            load_tile(c, G, base, S.fresh != 0);
            double a = 0;
            for (uint32_t i = tid; i < c.tsize; i += kWG) a += abs2d(c.L[i]);
            const double s = wg_sum1(c, a);
            if (tid == 0) tsums[t] = s;
        }
        if (tid == 0) {
            S.st[ST_PASSES] += 1;
            S.st[ST_BYTES] += S.fresh ? 0 : (1ull << n) * sizeof(A);
            double r2 = 0;  // tile sums -> inclusive prefix
            for (uint32_t t = 0; t < c.n_tiles; ++t) {
                r2 += tsums[t];
                tsums[t] = r2;
            }
        }
        __threadfence_block();
        __syncthreads();
    }
    const double N = tsums[c.n_tiles - 1];
    // tile of each shot -> shot_tmp[i]
    for (int i = S.lo + tid; i < S.hi; i += kWG) {
        const uint64_t shot = (uint64_t)P.shot_perm[i];
        const double x = philox_u01(P.seed, P.shot_base + shot, op.r, 0) * N;
        int t = -1;
        uint32_t lo = 0, hi = c.n_tiles;  // first t with x < tsums[t]
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (x < tsums[mid]) hi = mid; else lo = mid + 1;
        }
        if (lo < c.n_tiles) {
            t = (int)lo;
        } else {  // rounding: last tile with weight
            for (int tt = (int)c.n_tiles - 1; tt >= 0; --tt) {
                const double prev = tt ? tsums[tt - 1] : 0.0;
                if (tsums[tt] > prev) { t = tt; break; }
            }
            if (t < 0) t = 0;
        }
        P.shot_tmp[i] = t;
    }
    __threadfence_block();
    __syncthreads();
    for (uint32_t t = 0; t < c.n_tiles; ++t) {
        // does any shot land in tile t?
        if (tid == 0) S.anyhigh = 0;
        __syncthreads();
        for (int i = S.lo + tid; i < S.hi; i += kWG)
            if (P.shot_tmp[i] == (int)t) { S.anyhigh = 1; break; }
        __syncthreads();
        const int hit = S.anyhigh;
        __syncthreads();
        if (!hit) continue;
        if (!P.resident) {
            load_tile(c, G, (uint64_t)t << k, S.fresh != 0);
            tile_prefix();
        }
        const double excl = t ? tsums[t - 1] : 0.0;
        int ties = 0;
        for (int i = S.lo + tid; i < S.hi; i += kWG) {
            if (P.shot_tmp[i] != (int)t) continue;
            const uint64_t shot = (uint64_t)P.shot_perm[i];
            const double x = philox_u01(P.seed, P.shot_base + shot, op.r, 0) * N;
            uint32_t lo = 0, hi = c.tsize;  // first e with x < excl + D[e]
            while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                if (x < excl + D[mid]) hi = mid; else lo = mid + 1;
            }
            uint32_t e = lo;
            // margin: the tile boundaries that chose tile t, then the
            // in-tile boundaries that chose entry e (the last entry of the
            // state has no upper boundary)
            double mg = 0.0;
            if (e < c.tsize && x < tsums[t]) {
                const bool last_tile = t + 1 == c.n_tiles;
                mg = __builtin_inf();
                if (t > 0) mg = fmin(mg, x - excl);
                if (!last_tile) mg = fmin(mg, tsums[t] - x);
                if (e > 0) mg = fmin(mg, x - (excl + D[e - 1]));
                if (!(last_tile && e == c.tsize - 1)) mg = fmin(mg, excl + D[e] - x);
                mg = N > 0 ? mg / N : 0.0;
            }
            ties += note_margin(P, shot, mg);
            if (e >= c.tsize) {  // rounding: last non-zero entry of the tile
                e = c.tsize - 1;
                while (e > 0 && !(D[e] > D[e - 1])) --e;
            }
            const uint64_t idx = ((uint64_t)t << k) | e;
            uint64_t mm = creg_load(P.memory + shot);
            for (int q = 0; q < n; ++q) {
                uint64_t bit = (idx >> q) & 1u;
                const double pf = bit ? P.ro10 : P.ro01;
                if (pf > 0 && philox_u01(P.seed, P.shot_base + shot, op.r, 1u + q) < pf) bit ^= 1u;
                mm = (mm & ~(1ull << op.c[q])) | (bit << op.c[q]);
            }
            creg_store(P.memory + shot, mm);
        }
        if (ties) atomicAdd((unsigned long long *)&S.st[ST_NEARTIES], (unsigned long long)ties);
        __syncthreads();
    }
}

// Write the normalised state of this branch into P.dump (complex double).
template <class R>
__device__ __noinline__ void dump_state(Ctx<R> &c, const PassInfo &pi)
{
    using A = typename V2<R>::T;
    const ExecParams &P = c.P;
    lds<WgShared> &S = c.S;
    const int n = P.n_qubits, k = P.tile_q;
    double2 *out = (double2 *)P.dump;
    double a = 0;
    if (P.resident) {
        for (uint32_t i = c.tid; i < c.tsize; i += kWG) a += abs2d(c.L[i]);
        const double N = wg_sum1(c, a);
        const double f = 1.0 / sqrt(N);
        for (uint32_t i = c.tid; i < c.tsize; i += kWG) {
            const A v = c.L[i];
            out[i] = make_double2((double)v.x * f, (double)v.y * f);
        }
        __syncthreads();
        return;
    }
    gbl<A> *G = slot_ptr<R>(P, S.slot);
    build_hi_off(c, pi, k);
    for (uint32_t t = 0; t < c.n_tiles; ++t) {
        load_tile(c, G, tile_base<R>(pi, n, k, t), S.fresh != 0);
        for (uint32_t i = c.tid; i < c.tsize; i += kWG) a += abs2d(c.L[i]);
        __syncthreads();
    }
    const double N = wg_sum1(c, a);
    const double f = 1.0 / sqrt(N);
    for (uint32_t t = 0; t < c.n_tiles; ++t) {
        const uint64_t base = tile_base<R>(pi, n, k, t);
        load_tile(c, G, base, S.fresh != 0);
        for (uint32_t l = c.tid; l < c.tsize; l += kWG) {
            const uint64_t g = base + c.hi_off[l >> kCoalesceQ] + (l & kRunMask);
            const A v = c.L[l];
            out[g] = make_double2((double)v.x * f, (double)v.y * f);
        }
        __syncthreads();
    }
}

template <class R>
__device__ __noinline__ void maybe_dump(Ctx<R> &c, int at_op)
{
    const ExecParams &P = c.P;
    lds<WgShared> &S = c.S;
    if (P.dump_shot < 0 || P.dump == nullptr) return;
    if (c.tid == 0) S.dump_here = 0;
    __syncthreads();
    for (int i = S.lo + c.tid; i < S.hi; i += kWG)
        if ((int64_t)P.shot_perm[i] == P.dump_shot) S.dump_here = 1;
    __syncthreads();
    if (!S.dump_here) return;
    const int pidx = P.ops[at_op < P.n_ops ? at_op : P.n_ops - 1].pass;
    dump_state(c, P.passes[pidx]);
}

// Register budget: configurations whose tile lets two workgroups share a
// CU are held to two waves per SIMD (256 VGPRs), so one workgroup can
// stream its tile while the other computes.
template <class R, int NR>
constexpr int exec_waves() { return (NR > 0 && NR * (int)sizeof(R) * 2 <= 256) ? 2 : 1; }

// The persistent executor. MF: complex64 one-qubit micro-ops on the matrix
// cores (a separate instantiation, so the other form's loop keeps its code)
template <class R, int NR, bool MF>
__device__ __forceinline__ void exec_body(const ExecParams &P)
{
    using A = typename V2<R>::T;
    extern __shared__ __align__(16) unsigned char smem[];
    // no static LDS: the tile starts at LDS address 0 and the per-workgroup
    // state sits at the end of the dynamic allocation
    lds<unsigned char> *sm0 = (lds<unsigned char> *)smem;
    lds<WgShared> &S =
        *(lds<WgShared> *)(sm0 + svb_side_bytes_dev(P.tile_q, (int)sizeof(A), P.resident, P.nbuf));
    const int tid = threadIdx.x;
    const int n = P.n_qubits, k = P.tile_q;
    Ctx<R> c{P, S};
    c.tid = tid;
    c.k = k;
    c.swm = 0;
    c.tsize = 1u << k;
    c.n_tiles = P.resident ? 1u : (1u << (n - k));
    lds<unsigned char> *sm = sm0;
    c.L = (lds<A> *)sm;
    c.lbase = 0;
    c.hi_off = (lds<uint32_t> *)(sm + (size_t)c.tsize * sizeof(A) * (P.resident ? 1 : P.nbuf));
    const uint32_t n_hi = P.resident ? 4u : (1u << (k - kCoalesceQ));
    c.dec = (lds<int16_t> *)(c.hi_off + n_hi);
    lds<unsigned char> *uarea = (lds<unsigned char> *)(c.dec + kMaxPassOps);
    c.scr = uarea;
    // split counters live in the tile when it is streamed and large enough
    const bool cnt_in_tile = !P.resident && (size_t)c.tsize * sizeof(A) >= 16u * kWG * 4u;
    c.cnt = cnt_in_tile ? (lds<int> *)sm : (lds<int> *)uarea;
    c.ug = (lds<UGroup> *)uarea;
    c.uops = (lds<UOp> *)(uarea + kMaxPassGroups * sizeof(UGroup));
    c.mats = (lds<R> *)((lds<unsigned char> *)c.uops + kMaxPassUops * sizeof(UOp));
    {
        // op staging area after the per-workgroup state
        lds<unsigned char> *st = (lds<unsigned char> *)&S + shared_bytes16();
        c.sops = P.stage_cap > 0 ? (const DevOp *)(lds<DevOp> *)st : nullptr;
        c.smat = (lds<double> *)(st + (size_t)P.stage_cap * sizeof(DevOp));
        c.s0 = 0;
        c.scap = 0;
        lds<unsigned char> *sr = (lds<unsigned char> *)(c.smat + (size_t)P.stage_cap * 8);
        c.srules = P.stage_rules ? (const DevRule *)(lds<DevRule> *)sr : nullptr;
        c.sroff = (lds<int32_t> *)(sr + kStageRules * sizeof(DevRule));
        c.sthr = (lds<double> *)(sr + (kStageRules * sizeof(DevRule) + kStageRules * sizeof(int32_t) + 15) /
                                          16 * 16);
        if (P.stage_rules) stage_rules(c);
    }
    if (tid < ST_COUNT) S.st[tid] = 0;
    __syncthreads();

    for (;;) {
        if (tid == 0) {
            S.status = ST_EXIT;
            Control *ctl = P.ctl;
            if (ld_rlx(&ctl->error) == 0) {
                const uint32_t t = atomicAdd(&ctl->q_head, 1u);
                if (t < (uint32_t)P.queue_cap && (P.branch_mode || t < ctl->n_initial)) {
                    // progress watchdog: the wait may last as long as other
                    // workgroups keep completing sweeps (a long unsplit
                    // record, the tail of the run); it fails only after
                    // spin_limit ticks in which no workgroup progressed
                    unsigned long long t0 = wall_clock64();
                    uint32_t hb = ld_rlx(&ctl->heartbeat);
                    for (;;) {
                        // poll relaxed; one acquire fence once the record is published
                        if (ld_rlx(&P.ready[t])) {
                            __atomic_thread_fence(__ATOMIC_ACQUIRE);
                            const BranchRec q = P.queue[t];
                            S.rec.slot = q.slot;
                            S.rec.lo = q.lo;
                            S.rec.hi = q.hi;
                            S.rec.cursor = q.cursor;
                            S.rec.pending = q.pending;
                            S.rec.flags = q.flags;
                            S.rec.scale = q.scale;
                            S.rec.norm_lb = q.norm_lb;
                            S.status = ST_WORK;
                            break;
                        }
                        if (ld_rlx_i(&ctl->outstanding) <= 0) break;
                        const uint32_t hb2 = ld_rlx(&ctl->heartbeat);
                        if (hb2 != hb && !P.spin_elapsed) {
                            hb = hb2;
                            t0 = wall_clock64();
                        } else if (spin_expired(t0, P.spin_limit)) {
                            atomicOr(&ctl->error, kErrTimeout);
                            break;
                        }
                        __builtin_amdgcn_s_sleep(8);
                    }
                }
            }
        }
        __syncthreads();
        if (S.status == ST_EXIT) break;

        // ---- set up the branch's state
        if (tid == 0) {
            S.lo = S.rec.lo;
            S.hi = S.rec.hi;
            S.cursor = S.rec.cursor;
            S.pending = S.rec.pending;
            S.first_scale = S.rec.scale;
            S.norm_lb = S.rec.norm_lb;
            if (P.resident) {
                S.slot = S.rec.slot;
                S.fresh = (S.rec.slot < 0) || (S.rec.flags & 1);
            } else if (P.private_slots) {
                S.slot = blockIdx.x;
                S.fresh = 1;
            } else {
                S.slot = S.rec.slot;
                S.fresh = S.rec.flags & 1;
            }
        }
        __syncthreads();
        if (P.resident) {
            if (S.fresh) {
                for (uint32_t i = tid; i < c.tsize; i += kWG) {
                    A z;
                    z.x = (i == 0) ? (R)1 : (R)0;
                    z.y = 0;
                    c.L[i] = z;
                }
            } else {
                const gbl<A> *G = slot_ptr<R>(P, S.slot);
                for (uint32_t i = tid; i < c.tsize; i += kWG) c.L[i] = G[i];
            }
            __syncthreads();
            if (S.slot >= 0 && tid == 0) slot_push(P, S.slot);
            if (tid == 0) { S.slot = -1; S.fresh = 0; }
            __syncthreads();
        }

        // ---- run the op list
        for (;;) {
            plan_pass(c);
            const int stop = S.stop;
            if (stop == STOP_TERMINAL || stop == STOP_END) {
                if (S.end > S.start) run_sweep<R, NR, MF>(c, false);
                if (tid == 0) { S.cursor = S.end; S.pending = -1; }
                __syncthreads();
                maybe_dump(c, S.cursor);
                if (stop == STOP_TERMINAL) {
                    if (tid == 0) S.stop_op = S.cursor;
                    __syncthreads();
                    terminal_sample(c);
                }
                break;
            }
            if (stop == STOP_NONE && S.end == S.start) {  // no progress: give up
                if (tid == 0) atomicOr(&P.ctl->error, kErrState);
                break;
            }
            if (S.end > S.start || stop == STOP_REDUCE) run_sweep<R, NR, MF>(c, stop == STOP_REDUCE);
            if (stop == STOP_NONE) {
                if (tid == 0) { S.cursor = S.end; S.pending = -1; }
                __syncthreads();
                continue;
            }
            if (stop == STOP_REDUCE) {
                decide(c);
                continue;
            }
            // STOP_SPLIT on a Pauli channel
            split_branch(c, P.ops[S.stop_op], S.stop_op, S.split_cond != 0);
        }

        // ---- release the state and finish the record
        __syncthreads();
        if (tid == 0) {
            if (!P.resident && !P.private_slots && S.slot >= 0) slot_push(P, S.slot);
            __threadfence();
            __hip_atomic_fetch_add(&P.ctl->heartbeat, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            atomicSub(&P.ctl->outstanding, 1);
        }
        __syncthreads();
    }
    if (tid < ST_COUNT) atomicAdd(&P.ctl->stat[tid], S.st[tid]);
}

// The executor with complex64 one-qubit micro-ops on the matrix cores is
// compiled in kernels_mfma.hip (this file with SVB_MFMA_UNIT defined), so
// that its code does not share a code object with the default executor
template <class R, int NR>
__global__ void __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(exec_waves<R, NR>())))
exec_kernel_mfma(ExecParams P)
#ifdef SVB_MFMA_UNIT
{
    exec_body<R, NR, true>(P);
}
#else
    ;
#endif

#ifndef SVB_MFMA_UNIT
template <class R, int NR>
__global__ void __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(exec_waves<R, NR>())))
exec_kernel(ExecParams P)
{
    exec_body<R, NR, false>(P);
}

// Prepare one run (or one waiting-list relaunch).
__global__ void init_kernel(ExecParams P, int restart, int n_root_shots, int root_slot,
                            int n_free)
{
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int n_initial = P.branch_mode ? 1 : (int)P.n_shots;
    for (int64_t i = gid; i < P.n_shots; i += stride) {
        if (!restart) {
            P.memory[i] = 0;
            P.margins[i] = kInfBits;
            P.shot_perm[i] = (int32_t)i;
        }
    }
    for (int64_t i = gid; i < P.queue_cap; i += stride) {
        if (i < n_initial) {
            BranchRec r;
            if (P.branch_mode) {
                r.slot = root_slot;
                r.lo = 0;
                r.hi = n_root_shots;
            } else {
                r.slot = -1;
                r.lo = (int32_t)i;
                r.hi = (int32_t)i + 1;
            }
            r.cursor = 0;
            r.pending = -1;
            r.flags = 1;
            r.scale = 1.0;
            r.norm_lb = 1.0;
            P.queue[i] = r;
            P.ready[i] = 1u;
        } else {
            P.ready[i] = 0u;
        }
    }
    for (int64_t i = gid; i < n_free; i += stride) {
        // free stack: every slot except the root's
        P.free_slots[i] = (int32_t)((root_slot < 0 || i < root_slot) ? i : i + 1);
    }
    if (gid == 0) {
        Control *ctl = P.ctl;
        ctl->q_head = 0;
        ctl->q_tail = n_initial;
        ctl->outstanding = n_initial;
        ctl->error = 0;
        ctl->lock = 0;
        ctl->free_top = n_free;
        ctl->wait_count = 0;
        ctl->n_initial = n_initial;
        for (int s = 0; s < ST_COUNT; ++s) ctl->stat[s] = 0;
        ctl->done_workers = 0;
        ctl->heartbeat = 0;
    }
}

// Waiting-list relaunch: the parked shots become the root's range and
// their registers are cleared.
__global__ void restart_kernel(ExecParams P, int n_wait)
{
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = gid; i < n_wait; i += stride) {
        const int32_t s = P.waiting[i];
        P.shot_perm[i] = s;
        P.memory[s] = 0;
        P.margins[s] = kInfBits;
    }
}

#endif  // SVB_MFMA_UNIT
}  // namespace svb

#ifndef SVB_MFMA_UNIT
// ------------------------------------------------------------ launchers
// Executor instantiation: the matrix-core form exists for complex64 groups
// on two register sets (4 to 32 amplitudes per thread); 64 amplitudes per
// thread always run their one-qubit micro-ops on the matrix cores
template <class R, int NR>
static void *exec_entry(bool mfma)
{
    if constexpr (sizeof(R) == 4 && NR >= 4 && NR <= 32)
        if (mfma) return (void *)svb::exec_kernel_mfma<R, NR>;
    return (void *)svb::exec_kernel<R, NR>;
}

static size_t uarea_bytes(int cnt_in_tile)
{
    const size_t fuse = svb::kMaxPassGroups * sizeof(svb::UGroup) + svb::kMaxPassUops * sizeof(svb::UOp) +
                        svb::kPassMatBytes;
    const size_t cnt = 16 * svb::kWG * 4;  // split counters, unless they fit in the tile
    return (!cnt_in_tile && cnt > fuse) ? cnt : fuse;
}

extern "C" size_t svb_exec_lds_bytes(int tile_q, int amp_bytes, int resident, int nbuf,
                                     int stage_cap)
{
    const size_t tile = ((size_t)1 << tile_q) * amp_bytes;
    const size_t tiles = tile * (resident ? 1 : nbuf);
    const size_t hi = resident ? 4 * 4 : ((size_t)1 << (tile_q - svb::kCoalesceQ)) * 4;
    const size_t dec = svb::kMaxPassOps * 2;
    const int cnt_in_tile = !resident && tile >= 16u * svb::kWG * 4u;
    const size_t side = (tiles + hi + dec + uarea_bytes(cnt_in_tile) + 15) / 16 * 16;
    return side + svb::shared_bytes16() + svb::stage_bytes(stage_cap);
}

extern "C" {

hipError_t svb_launch_init(const svb::ExecParams *P, int restart, int n_root, int root_slot,
                           int n_free, hipStream_t st)
{
    hipLaunchKernelGGL(svb::init_kernel, dim3(1024), dim3(256), 0, st, *P, restart, n_root,
                       root_slot, n_free);
    return hipGetLastError();
}

// Kernel nodes of a graph-replayed run: function, grid, block and dynamic
// LDS of the initialisation kernel and of the executor instantiation that
// svb_launch_exec would launch (the executor's LDS attribute is set here).
hipError_t svb_graph_nodes(const svb::ExecParams *P, int is_c128, int reg_bits, int workers,
                           void **init_fn, unsigned *init_grid, void **exec_fn,
                           unsigned *exec_grid, unsigned *block, size_t *exec_lds)
{
    *init_fn = (void *)svb::init_kernel;
    *init_grid = 1024;
    *block = svb::kWG;
    *exec_grid = (unsigned)workers;
    *exec_lds = svb_exec_lds_bytes(P->tile_q, is_c128 ? 16 : 8, P->resident, P->nbuf, P->stage_cap);
    void *fn = nullptr;
#define SVB_FN(RT, N) fn = exec_entry<RT, N>(P->mfma1 != 0)
    if (is_c128) {
        if (reg_bits == 5) SVB_FN(double, 32);
        else if (reg_bits == 4) SVB_FN(double, 16);
        else if (reg_bits == 3) SVB_FN(double, 8);
        else if (reg_bits == 2) SVB_FN(double, 4);
        else SVB_FN(double, 0);
    } else {
        if (reg_bits == 6) SVB_FN(float, 64);
        else if (reg_bits == 5) SVB_FN(float, 32);
        else if (reg_bits == 4) SVB_FN(float, 16);
        else if (reg_bits == 3) SVB_FN(float, 8);
        else if (reg_bits == 2) SVB_FN(float, 4);
        else SVB_FN(float, 0);
    }
#undef SVB_FN
    *exec_fn = fn;
    return hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)*exec_lds);
}

hipError_t svb_launch_restart(const svb::ExecParams *P, int n_wait, hipStream_t st)
{
    hipLaunchKernelGGL(svb::restart_kernel, dim3(256), dim3(256), 0, st, *P, n_wait);
    return hipGetLastError();
}

}  // extern "C"

template <class R, int NR>
static hipError_t launch_one(const svb::ExecParams *P, int workers, size_t lds, hipStream_t st,
                             int *occ)
{
    const void *fn = exec_entry<R, NR>(P && P->mfma1);
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (occ) return hipOccupancyMaxActiveBlocksPerMultiprocessor(occ, fn, svb::kWG, lds);
    // launched by name with the argument by value (measured 0.6% faster on
    // the 20-qubit workload than through an argument-pointer array)
    if constexpr (sizeof(R) == 4 && NR >= 4 && NR <= 32) {
        if (fn == (const void *)svb::exec_kernel_mfma<R, NR>) {
            hipLaunchKernelGGL((svb::exec_kernel_mfma<R, NR>), dim3(workers), dim3(svb::kWG), lds, st,
                               *P);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((svb::exec_kernel<R, NR>), dim3(workers), dim3(svb::kWG), lds, st, *P);
    return hipGetLastError();
}

static hipError_t dispatch(const svb::ExecParams *P, int is_c128, int reg_bits, int tile_q,
                           int resident, int nbuf, int stage_cap, int workers, hipStream_t st,
                           int *occ)
{
    const size_t lds = svb_exec_lds_bytes(tile_q, is_c128 ? 16 : 8, resident, nbuf, stage_cap);
    if (is_c128) {
        if (reg_bits == 5) return launch_one<double, 32>(P, workers, lds, st, occ);
        if (reg_bits == 4) return launch_one<double, 16>(P, workers, lds, st, occ);
        if (reg_bits == 3) return launch_one<double, 8>(P, workers, lds, st, occ);
        if (reg_bits == 2) return launch_one<double, 4>(P, workers, lds, st, occ);
        return launch_one<double, 0>(P, workers, lds, st, occ);
    }
    if (reg_bits == 6) return launch_one<float, 64>(P, workers, lds, st, occ);
    if (reg_bits == 5) return launch_one<float, 32>(P, workers, lds, st, occ);
    if (reg_bits == 4) return launch_one<float, 16>(P, workers, lds, st, occ);
    if (reg_bits == 3) return launch_one<float, 8>(P, workers, lds, st, occ);
    if (reg_bits == 2) return launch_one<float, 4>(P, workers, lds, st, occ);
    return launch_one<float, 0>(P, workers, lds, st, occ);
}

extern "C" {

hipError_t svb_launch_exec(const svb::ExecParams *P, int is_c128, int reg_bits, int workers,
                           hipStream_t st)
{
    return dispatch(P, is_c128, reg_bits, P->tile_q, P->resident, P->nbuf, P->stage_cap, workers, st,
                    nullptr);
}

hipError_t svb_exec_occupancy(int is_c128, int tile_q, int resident, int reg_bits, int nbuf,
                              int stage_cap, int *blocks_per_cu)
{
    return dispatch(nullptr, is_c128, reg_bits, tile_q, resident, nbuf, stage_cap, 0, nullptr,
                    blocks_per_cu);
}

}  // extern "C"
#endif  // SVB_MFMA_UNIT
