/*
 * FP64 trajectory oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously-correct CPU reference for the multi-shot noisy
 * state-vector method of Doi, Horii and Wood, "Efficient techniques to GPU
 * Accelerations of Multi-Shot Quantum Computing Simulations" (arXiv
 * 2308.03399). Only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark may load it; the product library never does.
 *
 * Each shot is simulated on its own, from |0...0>, op by op, in double
 * precision: no batching, no branching, no fusion, no reordering. It shares
 * no code with the GPU library: its own op codes, noise-site expansion,
 * counter-based generator and gate loops.
 *
 * Readings of the paper taken here (the paper is silent or garbled there):
 *  - Kraus selection (Sec. III-B, Kraus pseudo-code): the chosen matrix is
 *    applied as K_j / sqrt(p_j) with p_j = ||K_j psi||^2 so the state stays
 *    normalised; the printed "matrix/p" would not.
 *  - Comparisons of a uniform u against a state-dependent running sum are
 *    made as u*N < S with N the squared norm from the same sweep (identical
 *    to u < S for a normalised state).
 *  - If rounding leaves every comparison false, the last candidate with a
 *    non-zero probability is taken.
 *  - Pauli channels (Sec. III-B, Table I): the listed probabilities are
 *    accumulated in list order and the first entry whose running sum
 *    exceeds u is taken (u strictly lower than the sum).
 *  - Measurement of qubits Q (Sec. IV-A, measure/reset pseudo-code):
 *    outcome i runs over 0..2^|Q|-1 with bit t of i the value of qubit
 *    Q[t]; the state collapses onto the chosen outcome and is renormalised;
 *    reset (alone or after a measure) then returns measured 1s to |0>.
 *  - Conditional operations (Sec. IV-A: conditional gates refer to measured
 *    classical bits, branch operations set a classical bit from them): an
 *    op with a non-zero condition mask runs only if (creg & mask) == value,
 *    and the noise channels attached to a conditional gate carry the same
 *    condition; a branch op sets its clbit to ((creg & mask) == value). A
 *    skipped op keeps its place in the op numbering (its draws are unused).
 *  - Readout error (named in Sec. III-B, no model given): each recorded bit
 *    flips independently, 0->1 with p01 and 1->0 with p10, from its own draw.
 *  - Decision margin (not an arithmetic step: a record of how close each
 *    state-dependent choice came to going the other way). For a Kraus or
 *    measure decision with running sums C_0 <= C_1 <= ... over n_c
 *    candidates, x = u*N and chosen index j, the margin is the distance
 *    from x to the nearest boundary that separates j from a neighbour:
 *    C_{j-1} if j > 0 and C_j if j < n_c - 1, divided by N; a choice made
 *    by the rounding fall-back has margin 0. Each shot reports the smallest
 *    margin of its decisions (+inf if it made none).
 *  - Random numbers: u = U(seed, shot, r, d) from Philox4x32-10 (Salmon,
 *    Moraes, Dror, Shaw, SC'11) with key = (seed lo, seed hi) and counter
 *    = (shot lo, shot hi, r, d); r is the op's index in the expanded list,
 *    d = 0 for the op's draw and 1 + t for the readout flip of bit t; the
 *    53-bit double is ((x0 >> 5) * 2^26 + (x1 >> 6)) * 2^-53.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* ------------------------------------------------------------------------ */
/* Op codes of the oracle's own input format                                 */
/* ------------------------------------------------------------------------ */
enum {
    O_ID = 0, O_X, O_Y, O_Z, O_H, O_S, O_SDG, O_T, O_TDG, O_U3,
    O_CX = 16, O_CZ, O_SWAP,
    O_UNITARY = 24,
    O_MEASURE = 32, O_RESET, O_MEASURE_RESET,
    O_BFUNC = 40,      /* clbit c[0] <- ((creg & cmask) == cval) */
    /* inserted by the noise expansion only */
    O_PAULI_CH = 48, O_KRAUS_CH
};

#define MAXQ 32   /* qubits (and clbits) per op */
#define MAXDENSE 5 /* qubits of a dense matrix */

typedef struct {
    int kind;
    int nq;
    int q[MAXQ];
    int c[MAXQ];
    double par[3];
    const double *mat; /* UNITARY / KRAUS matrices, interleaved re/im */
    int rule;          /* noise rule index for channel ops */
    uint64_t cmask;    /* condition (or branch-op predicate): (creg & cmask) == cval */
    uint64_t cval;
} xop;

typedef struct {
    unsigned gate_mask_lo; /* bit k set: gates of op code k (k < 32) */
    int type;              /* 0 pauli, 1 kraus */
    int nq;
    int n_terms;
    const double *prob;    /* pauli: n_terms probabilities */
    const int *codes;      /* pauli: n_terms rows of MAXQ codes, I0 X1 Y2 Z3 */
    const double *mats;    /* kraus: n_terms matrices (2^nq)^2 complex */
} xrule;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from the round function and key schedule published in      */
/* Salmon et al., SC'11 (multipliers 0xD2511F53, 0xCD9E8D57; Weyl key        */
/* increments 0x9E3779B9, 0xBB67AE85).                                       */
/* ------------------------------------------------------------------------ */
void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                          uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

double oracle_uniform(uint64_t seed, uint64_t shot, uint32_t r, uint32_t d)
{
    uint32_t ctr[4] = {(uint32_t)shot, (uint32_t)(shot >> 32), r, d};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t x[4];
    oracle_philox4x32_10(ctr, key, x);
    uint64_t hi = x[0] >> 5; /* 27 bits */
    uint64_t lo = x[1] >> 6; /* 26 bits */
    return (double)(hi * 67108864ull + lo) * (1.0 / 9007199254740992.0);
}

/* ------------------------------------------------------------------------ */
/* Gate matrices (textbook definitions; U3 as in OpenQASM 2)                 */
/* ------------------------------------------------------------------------ */
static void gate_matrix_1q(int kind, const double *par, cplx m[4])
{
    const double r2 = 1.0 / sqrt(2.0);
    switch (kind) {
    case O_ID: m[0] = 1; m[1] = 0; m[2] = 0; m[3] = 1; break;
    case O_X: m[0] = 0; m[1] = 1; m[2] = 1; m[3] = 0; break;
    case O_Y: m[0] = 0; m[1] = -I; m[2] = I; m[3] = 0; break;
    case O_Z: m[0] = 1; m[1] = 0; m[2] = 0; m[3] = -1; break;
    case O_H: m[0] = r2; m[1] = r2; m[2] = r2; m[3] = -r2; break;
    case O_S: m[0] = 1; m[1] = 0; m[2] = 0; m[3] = I; break;
    case O_SDG: m[0] = 1; m[1] = 0; m[2] = 0; m[3] = -I; break;
    case O_T: m[0] = 1; m[1] = 0; m[2] = 0; m[3] = cexp(I * M_PI / 4); break;
    case O_TDG: m[0] = 1; m[1] = 0; m[2] = 0; m[3] = cexp(-I * M_PI / 4); break;
    case O_U3: {
        double th = par[0], ph = par[1], la = par[2];
        double c = cos(th / 2), s = sin(th / 2);
        m[0] = c;
        m[1] = -cexp(I * la) * s;
        m[2] = cexp(I * ph) * s;
        m[3] = cexp(I * (ph + la)) * c;
        break;
    }
    default: abort();
    }
}

/* m is row-major over a 2-dim space: new[a] = sum_b m[a*2+b] old[b] */
static void apply_1q(cplx *psi, int n, int q, const cplx m[4])
{
    uint64_t dim = 1ull << n, bit = 1ull << q;
    for (uint64_t i = 0; i < dim; ++i) {
        if (i & bit) continue;
        cplx a = psi[i], b = psi[i | bit];
        psi[i] = m[0] * a + m[1] * b;
        psi[i | bit] = m[2] * a + m[3] * b;
    }
}

/* Dense k-qubit matrix on qubits qs[0..k-1]; bit t of the matrix index is
 * the value of qubit qs[t]. */
static void apply_dense(cplx *psi, int n, int k, const int *qs, const cplx *m)
{
    uint64_t dim = 1ull << n, sub = 1ull << k, mask = 0;
    for (int t = 0; t < k; ++t) mask |= 1ull << qs[t];
    cplx in[1 << MAXDENSE], out[1 << MAXDENSE];
    uint64_t idx[1 << MAXDENSE];
    if (k > MAXDENSE) abort();
    for (uint64_t base = 0; base < dim; ++base) {
        if (base & mask) continue;
        for (uint64_t a = 0; a < sub; ++a) {
            uint64_t j = base;
            for (int t = 0; t < k; ++t)
                if ((a >> t) & 1) j |= 1ull << qs[t];
            idx[a] = j;
            in[a] = psi[j];
        }
        for (uint64_t a = 0; a < sub; ++a) {
            cplx acc = 0;
            for (uint64_t b = 0; b < sub; ++b) acc += m[a * sub + b] * in[b];
            out[a] = acc;
        }
        for (uint64_t a = 0; a < sub; ++a) psi[idx[a]] = out[a];
    }
}

static void apply_cx(cplx *psi, int n, int c, int t)
{
    uint64_t dim = 1ull << n, cb = 1ull << c, tb = 1ull << t;
    for (uint64_t i = 0; i < dim; ++i) {
        if ((i & cb) && !(i & tb)) {
            cplx tmp = psi[i];
            psi[i] = psi[i | tb];
            psi[i | tb] = tmp;
        }
    }
}

static void apply_cz(cplx *psi, int n, int a, int b)
{
    uint64_t dim = 1ull << n, ab = 1ull << a, bb = 1ull << b;
    for (uint64_t i = 0; i < dim; ++i)
        if ((i & ab) && (i & bb)) psi[i] = -psi[i];
}

static void apply_swap(cplx *psi, int n, int a, int b)
{
    uint64_t dim = 1ull << n, ab = 1ull << a, bb = 1ull << b;
    for (uint64_t i = 0; i < dim; ++i) {
        if ((i & ab) && !(i & bb)) {
            uint64_t j = (i & ~ab) | bb;
            cplx tmp = psi[i];
            psi[i] = psi[j];
            psi[j] = tmp;
        }
    }
}

static double norm2(const cplx *psi, int n)
{
    uint64_t dim = 1ull << n;
    double s = 0;
    for (uint64_t i = 0; i < dim; ++i)
        s += creal(psi[i]) * creal(psi[i]) + cimag(psi[i]) * cimag(psi[i]);
    return s;
}

static void scale(cplx *psi, int n, double f)
{
    uint64_t dim = 1ull << n;
    for (uint64_t i = 0; i < dim; ++i) psi[i] *= f;
}

/* Relative decision margin (see the header): prev = C_{j-1} (unused when
 * j == 0), cur = C_j (unused when j is the last candidate). */
static double decision_margin(double x, double N, int j, int n_cand, double prev,
                              double cur, int fell_back)
{
    if (fell_back) return 0.0;
    double m = INFINITY;
    if (j > 0 && x - prev < m) m = x - prev;
    if (j < n_cand - 1 && cur - x < m) m = cur - x;
    return N > 0 ? m / N : 0.0;
}

static void note_margin(double *mmin, double m)
{
    if (mmin && m < *mmin) *mmin = m;
}

/* ------------------------------------------------------------------------ */
/* Noise channels                                                            */
/* ------------------------------------------------------------------------ */

/* Pauli channel (Sec. III-B and Table I): sample one Pauli string by
 * comparing u with the running sum of the listed probabilities, then apply
 * it as the plain Pauli matrices, one qubit at a time. */
static void pauli_channel(cplx *psi, int n, const xop *op, const xrule *ru,
                          double u)
{
    double run = 0.0;
    int chosen = ru->n_terms - 1;
    for (int j = 0; j < ru->n_terms; ++j) {
        run += ru->prob[j];
        if (u < run) { chosen = j; break; }
    }
    for (int t = 0; t < ru->nq; ++t) {
        int code = ru->codes[chosen * MAXQ + t];
        static const int kinds[4] = {O_ID, O_X, O_Y, O_Z};
        if (code == 0) continue;
        cplx m[4];
        gate_matrix_1q(kinds[code], NULL, m);
        apply_1q(psi, n, op->q[t], m);
    }
}

/* Kraus channel (Sec. III-B, Kraus pseudo-code): walk the matrices in
 * order, accumulate p_j = ||K_j psi||^2 and take the first j whose running
 * sum exceeds u*N; psi <- K_j psi / sqrt(p_j). Returns the chosen j. */
static int kraus_channel(cplx *psi, cplx *work, int n, const xop *op,
                         const xrule *ru, double u, double *mmin)
{
    uint64_t dim = 1ull << n;
    int k = ru->nq, sub = 1 << k;
    double N = norm2(psi, n);
    double run = 0.0, prev = 0.0;
    int chosen = -1, last_nonzero = -1;
    double p_chosen = 0.0;
    for (int j = 0; j < ru->n_terms; ++j) {
        const cplx *m = (const cplx *)(ru->mats + (size_t)j * sub * sub * 2);
        memcpy(work, psi, dim * sizeof(cplx));
        apply_dense(work, n, k, op->q, m);
        double p = norm2(work, n);
        if (p > 0) last_nonzero = j;
        prev = run;
        run += p;
        if (u * N < run) { chosen = j; p_chosen = p; break; }
    }
    note_margin(mmin, decision_margin(u * N, N, chosen < 0 ? last_nonzero : chosen,
                                      ru->n_terms, prev, run, chosen < 0));
    if (chosen < 0) {
        chosen = last_nonzero;
        const cplx *m = (const cplx *)(ru->mats + (size_t)chosen * sub * sub * 2);
        memcpy(work, psi, dim * sizeof(cplx));
        apply_dense(work, n, k, op->q, m);
        p_chosen = norm2(work, n);
    }
    memcpy(psi, work, dim * sizeof(cplx));
    scale(psi, n, 1.0 / sqrt(p_chosen));
    return chosen;
}

/* Measure (and reset) of qubits op->q[0..nq-1] (Sec. IV-A, measure/reset
 * pseudo-code). Returns the outcome pattern. */
static uint64_t measure(cplx *psi, int n, const xop *op, double u, double *mmin)
{
    uint64_t dim = 1ull << n;
    int m = op->nq;
    uint64_t n_out = 1ull << m;
    double *P = (double *)calloc(n_out, sizeof(double));
    for (uint64_t i = 0; i < dim; ++i) {
        uint64_t pat = 0;
        for (int t = 0; t < m; ++t) pat |= ((i >> op->q[t]) & 1ull) << t;
        P[pat] += creal(psi[i]) * creal(psi[i]) + cimag(psi[i]) * cimag(psi[i]);
    }
    double N = 0.0;
    for (uint64_t o = 0; o < n_out; ++o) N += P[o];
    double run = 0.0, prev = 0.0;
    int64_t chosen = -1, last_nonzero = -1;
    for (uint64_t o = 0; o < n_out; ++o) {
        if (P[o] > 0) last_nonzero = (int64_t)o;
        prev = run;
        run += P[o];
        if (u * N < run) { chosen = (int64_t)o; break; }
    }
    note_margin(mmin, decision_margin(u * N, N, (int)(chosen < 0 ? last_nonzero : chosen),
                                      n_out > 0x7fffffff ? 0x7fffffff : (int)n_out,
                                      prev, run, chosen < 0));
    if (chosen < 0) chosen = last_nonzero;
    double f = 1.0 / sqrt(P[chosen]);
    for (uint64_t i = 0; i < dim; ++i) {
        uint64_t pat = 0;
        for (int t = 0; t < m; ++t) pat |= ((i >> op->q[t]) & 1ull) << t;
        psi[i] = (pat == (uint64_t)chosen) ? psi[i] * f : 0.0;
    }
    free(P);
    return (uint64_t)chosen;
}

static void reset_measured(cplx *psi, int n, const xop *op, uint64_t outcome)
{
    cplx xm[4];
    gate_matrix_1q(O_X, NULL, xm);
    for (int t = 0; t < op->nq; ++t)
        if ((outcome >> t) & 1) apply_1q(psi, n, op->q[t], xm);
}

/* ------------------------------------------------------------------------ */
/* Noise-site expansion: after each gate, every rule listing the gate's kind */
/* (and acting on as many qubits) adds its channel on the gate's qubits, in  */
/* rule order.                                                               */
/* ------------------------------------------------------------------------ */
static int is_gate(int kind)
{
    return kind < O_MEASURE;  /* channels copy the gate's condition too */
}

static int expand(int n_ops, const xop *ops, int n_rules, const xrule *rules,
                  xop *out)
{
    int w = 0;
    for (int i = 0; i < n_ops; ++i) {
        if (out) out[w] = ops[i];
        ++w;
        if (!is_gate(ops[i].kind)) continue;
        for (int r = 0; r < n_rules; ++r) {
            if (!((rules[r].gate_mask_lo >> ops[i].kind) & 1u)) continue;
            if (rules[r].nq != ops[i].nq) continue;
            if (out) {
                xop ch = ops[i];
                ch.kind = rules[r].type == 0 ? O_PAULI_CH : O_KRAUS_CH;
                ch.rule = r;
                ch.mat = NULL;
                out[w] = ch;
            }
            ++w;
        }
    }
    return w;
}

/* ------------------------------------------------------------------------ */
/* One shot                                                                  */
/* ------------------------------------------------------------------------ */
static uint64_t run_shot(int n, int n_x, const xop *x, const xrule *rules,
                         double ro01, double ro10, uint64_t seed,
                         uint64_t shot, int stop_at, cplx *psi, cplx *work,
                         double *mmin)
{
    uint64_t dim = 1ull << n;
    memset(psi, 0, dim * sizeof(cplx));
    psi[0] = 1.0;
    uint64_t creg = 0;
    int end = (stop_at >= 0 && stop_at < n_x) ? stop_at : n_x;
    for (int r = 0; r < end; ++r) {
        const xop *op = &x[r];
        if (op->kind == O_BFUNC) {
            const uint64_t bit = (creg & op->cmask) == op->cval;
            creg = (creg & ~(1ull << op->c[0])) | (bit << op->c[0]);
            continue;
        }
        if (op->cmask && (creg & op->cmask) != op->cval) continue;
        switch (op->kind) {
        case O_CX: apply_cx(psi, n, op->q[0], op->q[1]); break;
        case O_CZ: apply_cz(psi, n, op->q[0], op->q[1]); break;
        case O_SWAP: apply_swap(psi, n, op->q[0], op->q[1]); break;
        case O_UNITARY: apply_dense(psi, n, op->nq, op->q, (const cplx *)op->mat); break;
        case O_PAULI_CH:
            pauli_channel(psi, n, op, &rules[op->rule],
                          oracle_uniform(seed, shot, (uint32_t)r, 0));
            break;
        case O_KRAUS_CH:
            kraus_channel(psi, work, n, op, &rules[op->rule],
                          oracle_uniform(seed, shot, (uint32_t)r, 0), mmin);
            break;
        case O_MEASURE:
        case O_MEASURE_RESET:
        case O_RESET: {
            uint64_t o = measure(psi, n, op,
                                 oracle_uniform(seed, shot, (uint32_t)r, 0), mmin);
            if (op->kind != O_RESET) {
                for (int t = 0; t < op->nq; ++t) {
                    uint64_t bit = (o >> t) & 1ull;
                    double pf = bit ? ro10 : ro01;
                    if (pf > 0 && oracle_uniform(seed, shot, (uint32_t)r,
                                                 (uint32_t)(1 + t)) < pf)
                        bit ^= 1ull;
                    creg = (creg & ~(1ull << op->c[t])) | (bit << op->c[t]);
                }
            }
            if (op->kind != O_MEASURE) reset_measured(psi, n, op, o);
            break;
        }
        default: {
            cplx m[4];
            gate_matrix_1q(op->kind, op->par, m);
            apply_1q(psi, n, op->q[0], m);
        }
        }
    }
    return creg;
}

/* ------------------------------------------------------------------------ */
/* Entry point (called through ctypes by the test-suite).                   */
/*                                                                          */
/* op arrays: kind[n_ops], nq[n_ops], q[n_ops*8], c[n_ops*8], par[n_ops*3], */
/* mat_off[n_ops] (offset in doubles into mats, -1 if none).                */
/* rules: gate_mask[n_rules], type, nq, n_terms, off (into probs/codes for  */
/* Pauli, into kmats (doubles) for Kraus).                                  */
/* shots[n_sel] -> memory[n_sel]. If state_out != NULL, the state of        */
/* shots[0] after the first stop_at expanded ops (all if < 0) is written.   */
/* If margin_out != NULL, margin_out[s] receives the smallest decision      */
/* margin of shot s (see the header).                                       */
/* Returns the expanded op count, or -1 on an input error.                  */
/* ------------------------------------------------------------------------ */
int oracle_run(int n, int n_ops, const int *kind, const int *nq,
               const int *q, const int *c, const double *par,
               const uint64_t *cmask, const uint64_t *cval,
               const long *mat_off, const double *mats, int n_rules,
               const unsigned *gate_mask, const int *rtype, const int *rnq,
               const int *rnterms, const long *roff, const double *probs,
               const int *codes, const double *kmats, double ro01,
               double ro10, uint64_t seed, long n_sel, const int64_t *shots,
               uint64_t *memory, int stop_at, double *state_out,
               int n_threads, double *margin_out)
{
    if (n < 1 || n > 30 || n_ops < 0) return -1;
    xop *ops = (xop *)calloc((size_t)n_ops + 1, sizeof(xop));
    xrule *rules = (xrule *)calloc((size_t)n_rules + 1, sizeof(xrule));
    for (int i = 0; i < n_ops; ++i) {
        ops[i].kind = kind[i];
        ops[i].nq = nq[i];
        if (nq[i] < 0 || nq[i] > MAXQ || (kind[i] == O_UNITARY && nq[i] > MAXDENSE)) {
            free(ops); free(rules); return -1;
        }
        for (int t = 0; t < MAXQ; ++t) {
            ops[i].q[t] = q[i * MAXQ + t];
            ops[i].c[t] = c[i * MAXQ + t];
        }
        for (int t = 0; t < nq[i]; ++t)
            if (ops[i].q[t] < 0 || ops[i].q[t] >= n) { free(ops); free(rules); return -1; }
        for (int t = 0; t < 3; ++t) ops[i].par[t] = par[i * 3 + t];
        ops[i].mat = mat_off[i] >= 0 ? mats + mat_off[i] : NULL;
        ops[i].rule = -1;
        ops[i].cmask = cmask[i];
        ops[i].cval = cval[i];
        if ((cval[i] & ~cmask[i]) != 0) { free(ops); free(rules); return -1; }
        if (kind[i] == O_BFUNC && (nq[i] != 0 || c[i * MAXQ] < 0 || c[i * MAXQ] > 63)) {
            free(ops); free(rules); return -1;
        }
    }
    for (int r = 0; r < n_rules; ++r) {
        if (rnq[r] < 1 || rnq[r] > MAXDENSE) { free(ops); free(rules); return -1; }
        rules[r].gate_mask_lo = gate_mask[r];
        rules[r].type = rtype[r];
        rules[r].nq = rnq[r];
        rules[r].n_terms = rnterms[r];
        if (rtype[r] == 0) {
            rules[r].prob = probs + roff[r];
            rules[r].codes = codes + roff[r] * MAXQ;
        } else {
            rules[r].mats = kmats + roff[r];
        }
    }
    int n_x = expand(n_ops, ops, n_rules, rules, NULL);
    xop *x = (xop *)calloc((size_t)n_x + 1, sizeof(xop));
    expand(n_ops, ops, n_rules, rules, x);

    uint64_t dim = 1ull << n;
    if (state_out && n_sel > 0) {
        cplx *psi = (cplx *)malloc(dim * sizeof(cplx));
        cplx *work = (cplx *)malloc(dim * sizeof(cplx));
        double mm = INFINITY;
        memory[0] = run_shot(n, n_x, x, rules, ro01, ro10, seed,
                             (uint64_t)shots[0], stop_at, psi, work, &mm);
        if (margin_out) margin_out[0] = mm;
        memcpy(state_out, psi, dim * sizeof(cplx));
        free(psi);
        free(work);
    } else {
#pragma omp parallel num_threads(n_threads > 0 ? n_threads : 1)
        {
            cplx *psi = (cplx *)malloc(dim * sizeof(cplx));
            cplx *work = (cplx *)malloc(dim * sizeof(cplx));
#pragma omp for schedule(dynamic, 1)
            for (long s = 0; s < n_sel; ++s) {
                double mm = INFINITY;
                memory[s] = run_shot(n, n_x, x, rules, ro01, ro10, seed,
                                     (uint64_t)shots[s], stop_at, psi, work, &mm);
                if (margin_out) margin_out[s] = mm;
            }
            free(psi);
            free(work);
        }
    }
    free(x);
    free(ops);
    free(rules);
    return n_x;
}
