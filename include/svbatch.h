/*
 * svbatch.h -- C ABI of the MI355X multi-shot noisy state-vector library.
 *
 * The library runs many shots of one noisy quantum circuit on one gfx950 GPU
 * and returns the bit-count histogram of the classical register, the problem
 * statement of Doi, Horii and Wood, "Efficient techniques to GPU
 * Accelerations of Multi-Shot Quantum Computing Simulations" (arXiv
 * 2308.03399), Sec. III-B: a circuit, a noise model and a shot count go in,
 * a bit-count array comes out. Inside one launch it applies the circuit's
 * gates to per-shot 2^n-amplitude state vectors, samples per-shot Pauli
 * noise (Sec. IV-A, Pauli batching), selects per-shot Kraus operators
 * (Sec. IV-A, Kraus batching), performs mid-circuit measure/reset
 * (Sec. IV-A, measure/reset) and, in branch mode, shares one state among
 * shots until a draw splits them (Sec. IV-B, shot-branching).
 *
 * Conventions shared by every call:
 *  - Every function returns sv_status; no C++ exception crosses the ABI.
 *    On failure, sv_last_error() returns a thread-local message.
 *  - Host pointers are borrowed for the duration of the call only; the
 *    library copies what it keeps. Device memory is NOT allocated by the
 *    library: the caller attaches one device arena (sv_batch_attach) whose
 *    size is given by sv_batch_footprint, and a HIP stream on which all work
 *    is enqueued.
 *  - Calls on one handle must be serialised by the caller. Different
 *    handles may be used from different threads.
 *  - Basis index bit q is the value of qubit q (little-endian). Amplitudes
 *    of a state are stored contiguously, shot after shot (Sec. IV-A, data
 *    structure).
 *  - Random numbers: every random decision of shot s at expanded-op index r
 *    uses U(seed, s, r, d) of Philox4x32-10 (key = seed, counter =
 *    (s lo, s hi, r, d)), so the result of a shot does not depend on the
 *    mode, batch size, branching or number of relaunches.
 */
#ifndef SVBATCH_H
#define SVBATCH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sv_batch sv_batch; /* opaque; freed by sv_batch_destroy */

typedef enum { SV_C64 = 0, SV_C128 = 1 } sv_dtype;

typedef enum {
    SV_OK = 0,
    SV_EINVAL = 1,        /* invalid argument, circuit or noise model     */
    SV_ENOMEM = 2,        /* arena too small (not even one state fits)    */
    SV_EDEVICE = 3,       /* HIP error, or a device-side failure flag     */
    SV_ESTATE = 4,        /* call out of order (e.g. run before attach)   */
    SV_EUNSUPPORTED = 5   /* valid request outside what is implemented    */
} sv_status;

typedef enum {
    SV_MODE_BATCH = 0,    /* every shot owns a state (Sec. IV-A)          */
    SV_MODE_BRANCH = 1,   /* shots share states until split (Sec. IV-B)   */
    SV_MODE_PLAIN = 2     /* one state, one kernel per op, device
                             decisions: the conventional per-shot form
                             of Sec. III-C                               */
} sv_mode;

/* Op kinds of sv_op.kind. Gates act on q[0..nq-1]; for CX q[0] is the
 * control; for SV_OP_UNITARY bit t of the matrix row/column index is the
 * value of qubit q[t]. */
typedef enum {
    SV_OP_ID = 1, SV_OP_X, SV_OP_Y, SV_OP_Z, SV_OP_H, SV_OP_S, SV_OP_SDG,
    SV_OP_T, SV_OP_TDG,
    SV_OP_U3 = 10,        /* p = {theta, phi, lambda}, OpenQASM 2 U3        */
    SV_OP_CX = 20, SV_OP_CZ, SV_OP_SWAP,
    SV_OP_UNITARY = 30,   /* 1 to 5 qubits, dense matrix in mat            */
    SV_OP_MEASURE = 40,   /* qubits -> clbits (Sec. IV-A measure)           */
    SV_OP_RESET,          /* measure without record, then back to |0>      */
    SV_OP_MEASURE_RESET,  /* measure -> clbits, then back to |0>           */
    SV_OP_BFUNC = 45      /* branch op (Sec. IV-A): no qubits; clbit c[0] is
                             set to ((creg & cond_mask) == cond_value)     */
} sv_op_kind;

#define SV_MAX_INLINE 8   /* qubits/clbits held inline in sv_op            */
#define SV_MAX_CLBITS 64

typedef struct {
    uint32_t kind;                  /* sv_op_kind                                  */
    uint32_t nq;                    /* number of qubits (and clbits for measures)  */
    uint32_t q[SV_MAX_INLINE];      /* qubits, used when nq <= SV_MAX_INLINE       */
    uint32_t c[SV_MAX_INLINE];      /* clbits of MEASURE / MEASURE_RESET           */
    double p[3];                    /* SV_OP_U3 angles                             */
    const double *mat;              /* SV_OP_UNITARY: (2^nq)^2 complex, row-major,
                                       interleaved re/im; copied during the call   */
    const uint32_t *q_ext;          /* qubits when nq > SV_MAX_INLINE, else NULL   */
    const uint32_t *c_ext;          /* clbits when nq > SV_MAX_INLINE, else NULL   */
    uint64_t cond_mask;             /* conditional op (Sec. IV-A): it runs, with the
                                       noise attached to it, only for shots whose
                                       register satisfies (creg & cond_mask) ==
                                       cond_value; 0 = unconditional. For
                                       SV_OP_BFUNC: the predicate it records.   */
    uint64_t cond_value;            /* bits outside cond_mask must be 0 (EINVAL) */
} sv_op;

/* Pauli channel (Sec. III-B, Table I): n_terms (probability, Pauli string)
 * entries. pauli[j*nq + t] is the code of term j on the gate's qubit t,
 * I=0 X=1 Y=2 Z=3. Probabilities must be >= 0 and sum to 1 within 1e-12;
 * the entry taken is the first whose running sum exceeds the draw. nq is
 * 1 to 5, at most 1024 terms. */
typedef struct {
    uint32_t nq, n_terms;
    const double *prob;
    const uint8_t *pauli;
} sv_pauli_channel;

/* Kraus channel (Sec. III-B, Kraus operator): n_mats matrices of
 * (2^nq)^2 complex entries, row-major, interleaved re/im, with
 * sum_j K_j^dagger K_j = I within 1e-10. nq is 1 to 5, at most 16
 * matrices. */
typedef struct {
    uint32_t nq, n_mats;
    const double *mats;
} sv_kraus_channel;

/* A noise rule is attached after every gate whose kind bit is set in
 * gate_kinds_mask (bit k <-> sv_op_kind k) and whose qubit count equals the
 * channel's nq, on the gate's qubits, in rule order (the all-qubit error
 * rules of the paper's noise-model example, Sec. III-B). */
typedef struct {
    uint64_t gate_kinds_mask;
    uint32_t is_kraus;              /* 0: channel is sv_pauli_channel*, 1: sv_kraus_channel* */
    const void *channel;
} sv_noise_rule;

/* Readout error (named in Sec. III-B): each recorded bit flips 0->1 with
 * readout_p01 and 1->0 with readout_p10, from its own draw d = 1 + t. */
typedef struct {
    uint32_t n_rules;
    const sv_noise_rule *rules;
    double readout_p01, readout_p10;
} sv_noise_model;

typedef struct {
    double kernel_ms;          /* device time of the last run (HIP events)         */
    uint64_t passes;           /* state passes executed (tile sweeps of a state)   */
    uint64_t amp_bytes;        /* algorithmic bytes: passes * 2 * 2^n * amp size
                                  plus read-only reduction sweeps and copies       */
    uint64_t reductions;       /* FP64 reductions deciding Kraus/measure ops       */
    uint64_t branches;         /* states created by splits (branch mode)           */
    uint64_t restarts;         /* waiting-list relaunches (branch mode)            */
    uint64_t waiting_shots;    /* shots parked on the waiting list, summed         */
    uint64_t expanded_ops;     /* ops after noise-site expansion                   */
    uint64_t gate_count;       /* original gates (metric numerator per shot)       */
    uint32_t workers;          /* persistent workgroups launched                   */
    uint32_t slots;            /* state slots in the arena                         */
    uint32_t tile_qubits;      /* qubits per LDS tile                              */
    uint32_t static_passes;    /* passes of the static plan                        */
    uint64_t flops;            /* flops of the applied (fused) ops                 */
    double exec_ms;            /* device time of the executor launches only        */
    uint32_t exec_launches;    /* executor launches (1 + waiting-list relaunches)   */
    uint32_t tile_buffers;     /* LDS tile buffers of streamed grouped passes (1|2) */
    uint64_t groups;           /* register groups executed per sweep, summed       */
    uint64_t uops;             /* register micro-ops executed per sweep, summed    */
    uint64_t near_ties;        /* state-dependent decisions (Kraus, measure, final
                                  sample) whose relative margin is below 1e-9:
                                  see sv_get_margins                               */
    uint32_t graph_replays;    /* 1 if the run's initialisation and executor
                                  launches were replayed from the handle's HIP
                                  graph (option "graph"), else 0                   */
    uint32_t program_uploads;  /* 1 if the op program was copied to the device
                                  (0: unchanged since the last graph run)          */
    uint32_t mfma;             /* 1 if fused one-qubit micro-ops of complex64
                                  register groups ran on the matrix cores
                                  (option "mfma")                                  */
} sv_stats;

/* Create a handle for n_qubits (1..30) and n_shots (>= 1) in the given
 * storage dtype: the per-shot state vectors of 2^n_qubits amplitudes that
 * the batched execution of Sec. IV-A keeps for all shots (Sec. IV-A, data
 * structure), complex64 or complex128. No device work; the handle owns no
 * device memory until sv_batch_attach. SV_EINVAL on bad sizes or dtype;
 * *out is NULL on failure. */
sv_status sv_batch_create(int n_qubits, int64_t n_shots, sv_dtype dtype,
                          sv_batch **out);

/* Options (call before sv_batch_attach; some also between runs):
 *   "mode"         sv_mode                                   (default BATCH)
 *   "slots"        state slots in the arena; 0 = automatic (batch mode: one
 *                  per workgroup; branch mode: one per shot while they fit
 *                  in half the device memory free at sizing time, and at
 *                  least two per workgroup; fewer slots send shots to the
 *                  waiting list)
 *   "workers"      persistent workgroups; 0 = automatic (fills the GPU; in
 *                  batch mode, where each holds one state, at most as many
 *                  states as fit in 80% of the device memory free at sizing)
 *   "tile_qubits"  qubits per LDS tile, 6..14; 0 = automatic
 *   "pipeline"     LDS tile buffers of streamed states: -1 automatic (one,
 *                  with two workgroups per compute unit), 0 one, 1 two (the
 *                  next tile is fetched while the current one computes)
 *   "engine"       0 automatic (register groups for streamed states and
 *                  for resident states of 10 or more qubits up to 32 KiB;
 *                  one LDS sweep per op otherwise), 1 LDS sweeps everywhere,
 *                  2 register groups for every resident state of 10 or
 *                  more qubits
 *   "program_bytes" device bytes reserved for the op program (default 8 MiB)
 *   "dump_shot"    shot id whose state before the final op is kept for
 *                  sv_get_state; -1 disables (default)
 *   "spin_limit_ms" progress watchdog of the work queue (default 300000): a
 *                  workgroup waiting for a record gives up, and the run
 *                  fails with SV_EDEVICE, once this long has passed with no
 *                  workgroup completing a sweep or a record. A wait may
 *                  last as long as other workgroups keep progressing (a
 *                  long unsplit record, the tail of a run)
 *   "spin_elapsed" 1: the bound above counts from the start of each wait,
 *                  whatever the other workgroups do (forces the failure
 *                  path from the host in tests); 0 (default): watchdog
 *   "mfma"         complex64 fused one-qubit micro-ops: 0 automatic (the
 *                  matrix cores), 1 vector ALU, 2 matrix cores. Results
 *                  differ only by rounding
 *   "graph"        1: a run's two launches (initialisation, then the
 *                  persistent executor) are kept as a HIP graph on the handle;
 *                  later runs update the launch arguments (seed, shot offset,
 *                  program) and replay it, and skip the program upload when
 *                  the program is unchanged. Waiting-list relaunches (branch
 *                  mode) run outside the graph. 0 (default): direct launches
 *   "shot_offset"  global id of shot 0 (default 0): shot i of the handle draws
 *                  the randoms of global shot shot_offset + i, so a large job
 *                  can run as consecutive waves, or be split across devices,
 *                  with the same per-shot results
 * SV_EINVAL on an unknown key or bad value, SV_ESTATE if already attached
 * for keys that change the footprint. */
sv_status sv_batch_set_option(sv_batch *b, const char *key, int64_t value);

/* Device bytes the arena must hold for the current options, and the bytes
 * of one state (2^n * 8 for C64, 2^n * 16 for C128). Needs a visible GPU to
 * size the worker count. */
sv_status sv_batch_footprint(const sv_batch *b, uint64_t *bytes_required,
                             uint64_t *bytes_per_state);

/* Attach a caller-owned device buffer (at least sv_batch_footprint bytes,
 * 256-byte aligned) and the hipStream_t all work is enqueued on (NULL: the
 * null stream). The arena stays owned by the caller and must outlive the
 * handle's use. SV_ENOMEM if too small. */
sv_status sv_batch_attach(sv_batch *b, void *device_arena, uint64_t arena_bytes,
                          void *hip_stream);

/* Run all shots of the circuit ops[0..n_ops-1] under the noise model nm
 * (NULL: noiseless) with Philox seed `seed`: the multi-shot noise
 * simulation of Sec. III-B (a circuit, a noise model and a shot count in,
 * one classical register per shot out), executed as batched shots
 * (Sec. IV-A), shot-branching (Sec. IV-B) or the plain per-shot form
 * (Sec. III-C) according to the "mode" option. Validates first (qubits < n and
 * distinct within an op, clbits < 64, probabilities, Kraus completeness):
 * SV_EINVAL without touching the device. Blocks until the device work of
 * the run has finished. On any failure the handle is left in a state where
 * results are unavailable until the next successful run. A circuit without
 * ops (n_ops == 0) is valid: every shot's register is 0 and the state stays
 * |0..0>. */
sv_status sv_run_circuit(sv_batch *b, const sv_op *ops, size_t n_ops,
                         const sv_noise_model *nm, uint64_t seed);

/* Parameter sweep in one launch: n_sets circuits that differ only in the
 * angles of their U3 gates (the batched execution of Sec. IV-A, with the
 * per-state gate parameters of its parameter buffers varying by set).
 * params holds n_sets rows of 3 * n_u3 doubles, (theta, phi, lambda) of each
 * U3 op of ops[] in order; the p[] of those ops is ignored. The run's shots
 * are split evenly: set s owns shot ids [s*S/n_sets, (s+1)*S/n_sets), and
 * each of those shots is exactly the shot of sv_run_circuit on the circuit
 * with set s's angles. Batch mode only (SV_EUNSUPPORTED otherwise);
 * SV_EINVAL if n_sets is 0 or does not divide the shot count. Results as for
 * sv_run_circuit (memory in shot order, counts over all sets). */
sv_status sv_run_sweep(sv_batch *b, const sv_op *ops, size_t n_ops,
                       const sv_noise_model *nm, uint64_t seed,
                       const double *params, size_t n_sets);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc. The run of
 * sv_run_circuit, with the same results, on a device buffer the library
 * owns instead of an attached arena: a file-scope array of
 * SV_NOALLOC_MAX_BYTES on every GPU the library runs on, held from module
 * load until the process ends. The call allocates nothing (no hipMalloc,
 * hipFree or allocating library routine). b must not be attached
 * (SV_ESTATE); the work is enqueued on hip_stream (NULL: the null stream)
 * and the call blocks until it is done, then writes the n_memory == n_shots
 * per-shot registers to memory_out (host). The state slots are fitted to
 * the buffer (batch mode: as many workgroups as states fit); a run that
 * does not fit with one state slot fails with SV_ENOMEM and a message
 * giving the bytes it needs. Only sv_get_stats stays valid afterwards:
 * counts, margins and state dumps are not kept. Every call on one GPU
 * shares that GPU's buffer: calls that overlap on one GPU (other threads,
 * other handles) race and must be serialised by the caller. */
#define SV_NOALLOC_MAX_BYTES (64ull << 20)
sv_status sv_run_circuit_noalloc(sv_batch *b, const sv_op *ops, size_t n_ops,
                                 const sv_noise_model *nm, uint64_t seed,
                                 void *hip_stream, uint64_t *memory_out,
                                 size_t n_memory);

/* Bit-count histogram of the last run (Sec. III-B): keys[i] is a classical
 * register value (clbit c <-> bit c), counts[i] its number of shots, keys
 * ascending. If capacity < the number of distinct keys, *n_unique receives
 * the required size and SV_EINVAL is returned. */
sv_status sv_sample_counts(sv_batch *b, uint64_t *keys, uint64_t *counts,
                           size_t capacity, size_t *n_unique);

/* Per-shot classical registers of the last run ("memory"), shot order;
 * n must equal the shot count. */
sv_status sv_get_memory(sv_batch *b, uint64_t *creg_per_shot, size_t n);

/* Per-shot decision margins of the last run, shot order; n must equal the
 * shot count. A Kraus or measure choice compares u*N with the running sums
 * C_0 <= C_1 <= ... of its candidates (Sec. III-B Kraus pseudo-code,
 * Sec. IV-A measure pseudo-code; the final measurement samples the same way
 * over all 2^n outcomes). Its margin is the distance from u*N to the
 * boundaries that separate the chosen candidate j from its neighbours
 * (C_{j-1} if j > 0, C_j if j is not the last candidate), divided by N; a
 * choice made by the rounding fall-back has margin 0. out[s] is the
 * smallest margin of shot s, +inf if it made no such choice. Choices that
 * need no state (Pauli draws, readout flips, Kraus draws below the smallest
 * eigenvalue of K_0^dagger K_0) compare with host constants and are not
 * counted. Two exact implementations can disagree on a shot only where its
 * margin is of the order of their rounding error. */
sv_status sv_get_margins(sv_batch *b, double *margins, size_t n);

/* State of shot "dump_shot" before the last op of the circuit (normalised,
 * interleaved re/im doubles, 2^n complex). SV_ESTATE if none was kept. */
sv_status sv_get_state(sv_batch *b, double *amps, size_t n_amps);

/* Statistics of the last run (sv_stats above): device times, state passes
 * and the algorithmic bytes they move, reductions, branches and waiting-list
 * restarts (Sec. IV-B), near-ties. Valid after a successful run, also one of
 * sv_run_circuit_noalloc. SV_ESTATE before any. */
sv_status sv_get_stats(sv_batch *b, sv_stats *out);

/* Free the handle (host memory only; the attached arena stays the
 * caller's). NULL is accepted. */
sv_status sv_batch_destroy(sv_batch *b);

/* Message of the last failing call on this thread (static storage of the
 * thread, valid until its next failing call). */
const char *sv_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SVBATCH_H */
