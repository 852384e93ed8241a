// Plain per-shot form: the conventional GPU execution the batched and
// branched forms are measured against (Sec. III-C, the "GPU: Base" runs of
// Sec. V-B). One shot at a time, one kernel launch per op over the whole
// state, no batching, no fusion, no branching. Random decisions are taken
// on the device by a one-workgroup kernel per random op (FP64 sums of the
// per-block partials in a fixed order, the same Philox draws as the other
// modes), so the per-shot results equal those of batch and branch mode.
#include <hip/hip_runtime.h>
#include <algorithm>
#include <stdint.h>

#include "program.h"

namespace svb {
namespace plain {

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <class R> struct V2;
template <> struct V2<float> { using T = f32x2; };
template <> struct V2<double> { using T = f64x2; };

constexpr int kB = 256;       // threads per block
constexpr int kRed = 17;      // norm + 16 candidates

// Philox4x32-10 (Salmon et al., SC'11), as in the executor.
__device__ double philox_u01(uint64_t seed, uint64_t shot, uint32_t r, uint32_t d)
{
    uint32_t x0 = (uint32_t)shot, x1 = (uint32_t)(shot >> 32), x2 = r, x3 = d;
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
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

__device__ __forceinline__ uint64_t ins0(uint64_t p, uint32_t b)
{
    const uint64_t lo = p & ((1ull << b) - 1ull);
    return ((p ^ lo) << 1) | lo;
}

// decision cell written by a decide kernel, read by the apply kernel
struct Cell {
    int32_t outcome;
    int32_t pad;
    double scale;
};

template <class A, class R>
__device__ __forceinline__ A cmv(const double *m, double s, A a, A b, int row)
{
    const R m0r = (R)(m[4 * row] * s), m0i = (R)(m[4 * row + 1] * s);
    const R m1r = (R)(m[4 * row + 2] * s), m1i = (R)(m[4 * row + 3] * s);
    A o;
    o.x = m0r * a.x - m0i * a.y + m1r * b.x - m1i * b.y;
    o.y = m0r * a.y + m0i * a.x + m1r * b.y + m1i * b.x;
    return o;
}

template <class R>
__global__ void k_init(typename V2<R>::T *st, uint64_t namps, uint64_t *mem, uint64_t *marg)
{
    const uint64_t i = (uint64_t)blockIdx.x * kB + threadIdx.x;
    if (i < namps) {
        typename V2<R>::T z;
        z.x = i == 0 ? (R)1 : (R)0;
        z.y = 0;
        st[i] = z;
    }
    if (i == 0) {
        *mem = 0;
        *marg = kInfBits;
    }
}

// 2x2 matrix on qubit q (matrix m, or the decided Kraus matrix when cell)
template <class R>
__global__ void k_mat1(typename V2<R>::T *st, uint64_t npairs, uint32_t q, const double *m,
                       const Cell *cell, uint32_t mat_stride)
{
    using A = typename V2<R>::T;
    const uint64_t p = (uint64_t)blockIdx.x * kB + threadIdx.x;
    if (p >= npairs) return;
    double s = 1.0;
    if (cell) {
        m += (size_t)cell->outcome * mat_stride;
        s = cell->scale;
    }
    const uint64_t i0 = ins0(p, q), i1 = i0 | (1ull << q);
    const A a = st[i0], b = st[i1];
    st[i0] = cmv<A, R>(m, s, a, b, 0);
    st[i1] = cmv<A, R>(m, s, a, b, 1);
}

// Dense 2^NQ x 2^NQ matrix on qubits q[0..NQ-1] (bit t of its row/column
// index is qubit q[t]); the decided Kraus matrix when cell. One thread per
// base index: it holds the 2^NQ amplitudes and writes each output row.
template <class R, int NQ>
__global__ void k_dense(typename V2<R>::T *st, uint64_t nbase, const DevOp *op, const double *m,
                        const Cell *cell, uint32_t mat_stride)
{
    using A = typename V2<R>::T;
    constexpr int D = 1 << NQ;
    const uint64_t p = (uint64_t)blockIdx.x * kB + threadIdx.x;
    if (p >= nbase) return;
    double s = 1.0;
    if (cell) {
        m += (size_t)cell->outcome * mat_stride;
        s = cell->scale;
    }
    uint32_t q[NQ], sorted[NQ];
    for (int t = 0; t < NQ; ++t) q[t] = sorted[t] = op->q[t];
    for (int i = 0; i < NQ; ++i)
        for (int j = 0; j + 1 < NQ - i; ++j)
            if (sorted[j] > sorted[j + 1]) {
                const uint32_t t = sorted[j];
                sorted[j] = sorted[j + 1];
                sorted[j + 1] = t;
            }
    uint64_t base = p;
    for (int t = 0; t < NQ; ++t) base = ins0(base, sorted[t]);
    A v[D];
    for (int a = 0; a < D; ++a) {
        uint64_t idx = base;
        for (int t = 0; t < NQ; ++t) idx |= (uint64_t)((a >> t) & 1) << q[t];
        v[a] = st[idx];
    }
    for (int a = 0; a < D; ++a) {
        R xr = 0, xi = 0;
        for (int b = 0; b < D; ++b) {
            const R mr = (R)(m[2 * (D * a + b)] * s), mi = (R)(m[2 * (D * a + b) + 1] * s);
            xr += mr * v[b].x - mi * v[b].y;
            xi += mr * v[b].y + mi * v[b].x;
        }
        uint64_t idx = base;
        for (int t = 0; t < NQ; ++t) idx |= (uint64_t)((a >> t) & 1) << q[t];
        A o;
        o.x = xr;
        o.y = xi;
        st[idx] = o;
    }
}

template <class R>
static void launch_dense(typename V2<R>::T *st, int n, int nq, const DevOp *op, const double *m,
                         const Cell *cell, uint32_t mat_stride, hipStream_t stream)
{
    const uint64_t nbase = (1ull << n) >> nq;
    const dim3 g((unsigned)((nbase + kB - 1) / kB)), b(kB);
    switch (nq) {
    case 2: hipLaunchKernelGGL((k_dense<R, 2>), g, b, 0, stream, st, nbase, op, m, cell, mat_stride); break;
    case 3: hipLaunchKernelGGL((k_dense<R, 3>), g, b, 0, stream, st, nbase, op, m, cell, mat_stride); break;
    case 4: hipLaunchKernelGGL((k_dense<R, 4>), g, b, 0, stream, st, nbase, op, m, cell, mat_stride); break;
    default: hipLaunchKernelGGL((k_dense<R, 5>), g, b, 0, stream, st, nbase, op, m, cell, mat_stride); break;
    }
}

// CX (kind 0), CZ (1), SWAP (2)
template <class R>
__global__ void k_perm(typename V2<R>::T *st, uint64_t nquads, uint32_t q0, uint32_t q1, int kind)
{
    using A = typename V2<R>::T;
    const uint64_t p = (uint64_t)blockIdx.x * kB + threadIdx.x;
    if (p >= nquads) return;
    const uint32_t lo = q0 < q1 ? q0 : q1, hi = q0 < q1 ? q1 : q0;
    const uint64_t base = ins0(ins0(p, lo), hi);
    if (kind == 0) {
        const uint64_t i = base | (1ull << q0), j = i | (1ull << q1);
        const A t = st[i];
        st[i] = st[j];
        st[j] = t;
    } else if (kind == 1) {
        const uint64_t i = base | (1ull << q0) | (1ull << q1);
        A t = st[i];
        t.x = -t.x;
        t.y = -t.y;
        st[i] = t;
    } else {
        const uint64_t i = base | (1ull << q0), j = base | (1ull << q1);
        const A t = st[i];
        st[i] = st[j];
        st[j] = t;
    }
}

// Pauli channel draw (one thread)
__global__ void k_pauli_decide(uint64_t seed, uint64_t shot, uint32_t r, const double *thr,
                               int n_terms, Cell *cell)
{
    const double u = philox_u01(seed, shot, r, 0);
    int j = n_terms - 1;
    for (int t = 0; t < n_terms; ++t)
        if (u < thr[t]) { j = t; break; }
    cell->outcome = j;
    cell->scale = 1.0;
}

// Apply the drawn Pauli string (x/z masks over physical qubits, phase
// (-i)^ny); nothing to do for the identity.
template <class R>
__global__ void k_pauli_apply(typename V2<R>::T *st, uint64_t namps, const DevRule *ru,
                              const double *pool, const DevOp *op, const Cell *cell)
{
    using A = typename V2<R>::T;
    const int d = cell->outcome;
    const uint32_t code = (uint32_t)pool[ru->codes + (uint32_t)d];  // x | z << 8 | ny << 16
    if (code == 0) return;  // identity
    uint64_t xm = 0, zm = 0;
    for (int t = 0; t < op->nq; ++t) {
        xm |= (uint64_t)((code >> t) & 1u) << op->q[t];
        zm |= (uint64_t)((code >> (8 + t)) & 1u) << op->q[t];
    }
    const uint32_t ny = (code >> 16) & 3u;
    const uint64_t i = (uint64_t)blockIdx.x * kB + threadIdx.x;
    if (i >= namps) return;
    auto ph = [&](A v, uint64_t idx) {
        if (__popcll(idx & zm) & 1) { v.x = -v.x; v.y = -v.y; }
        A o;
        switch (ny) {
        case 0: o = v; break;
        case 1: o.x = v.y; o.y = -v.x; break;
        case 2: o.x = -v.x; o.y = -v.y; break;
        default: o.x = -v.y; o.y = v.x; break;
        }
        return o;
    };
    if (xm == 0) {
        st[i] = ph(st[i], i);
        return;
    }
    const uint64_t j = i ^ xm;
    if (i < j) {
        const A a = st[i], b = st[j];
        st[i] = ph(b, i);
        st[j] = ph(a, j);
    }
}

// Per-block partial sums of the norm and candidate weights of op (Kraus:
// ||K_j v||^2 over pairs/quads; measure: outcome probabilities).
template <class R>
__global__ void k_reduce(const typename V2<R>::T *st, int n, const DevOp *op, const DevRule *rules,
                         const double *pool, double *partial)
{
    using A = typename V2<R>::T;
    __shared__ double sh[kRed][kB / 64];
    double acc[kRed];
    for (int v = 0; v < kRed; ++v) acc[v] = 0;
    const uint64_t namps = 1ull << n;
    const uint64_t stride = (uint64_t)gridDim.x * kB;
    const uint64_t gid = (uint64_t)blockIdx.x * kB + threadIdx.x;
    if (op->kind == DK_KRAUS) {
        const DevRule &ru = rules[op->rule];
        const double *K = pool + ru.mats;
        const int nm = (int)ru.n_terms;
        if (ru.nq == 1) {
            const uint32_t q = op->q[0];
            for (uint64_t p = gid; p < namps / 2; p += stride) {
                const uint64_t i0 = ins0(p, q), i1 = i0 | (1ull << q);
                const A a = st[i0], b = st[i1];
                const double ar = a.x, ai = a.y, br = b.x, bi = b.y;
                acc[0] += ar * ar + ai * ai + br * br + bi * bi;
                for (int j = 0; j < nm && j < kMaxKraus; ++j) {
                    const double *m = K + j * 8;
                    const double w0r = m[0] * ar - m[1] * ai + m[2] * br - m[3] * bi;
                    const double w0i = m[0] * ai + m[1] * ar + m[2] * bi + m[3] * br;
                    const double w1r = m[4] * ar - m[5] * ai + m[6] * br - m[7] * bi;
                    const double w1i = m[4] * ai + m[5] * ar + m[6] * bi + m[7] * br;
                    acc[1 + j] += w0r * w0r + w0i * w0i + w1r * w1r + w1i * w1i;
                }
            }
        } else {
            const int nq = (int)ru.nq, D = 1 << nq;
            uint32_t q[kMaxDenseQ], sorted[kMaxDenseQ];
            for (int t = 0; t < nq; ++t) q[t] = sorted[t] = op->q[t];
            for (int i = 0; i < nq; ++i)
                for (int j = 0; j + 1 < nq - i; ++j)
                    if (sorted[j] > sorted[j + 1]) {
                        const uint32_t t = sorted[j];
                        sorted[j] = sorted[j + 1];
                        sorted[j + 1] = t;
                    }
            for (uint64_t p = gid; p < (namps >> nq); p += stride) {
                uint64_t base = p;
                for (int t = 0; t < nq; ++t) base = ins0(base, sorted[t]);
                double vr[1 << kMaxDenseQ], vi[1 << kMaxDenseQ];
                for (int a = 0; a < D; ++a) {
                    uint64_t idx = base;
                    for (int t = 0; t < nq; ++t) idx |= (uint64_t)((a >> t) & 1) << q[t];
                    const A v = st[idx];
                    vr[a] = v.x;
                    vi[a] = v.y;
                    acc[0] += vr[a] * vr[a] + vi[a] * vi[a];
                }
                for (int j = 0; j < nm && j < kMaxKraus; ++j) {
                    const double *m = K + (size_t)j * D * D * 2;
                    double sj = 0;
                    for (int a = 0; a < D; ++a) {
                        double wr = 0, wi = 0;
                        for (int b = 0; b < D; ++b) {
                            const double mr = m[2 * (D * a + b)], mi = m[2 * (D * a + b) + 1];
                            wr += mr * vr[b] - mi * vi[b];
                            wi += mr * vi[b] + mi * vr[b];
                        }
                        sj += wr * wr + wi * wi;
                    }
                    acc[1 + j] += sj;
                }
            }
        }
    } else {
        for (uint64_t i = gid; i < namps; i += stride) {
            uint32_t pat = 0;
            for (int t = 0; t < op->nq; ++t) pat |= (uint32_t)((i >> op->q[t]) & 1ull) << t;
            const A v = st[i];
            const double w = (double)v.x * v.x + (double)v.y * v.y;
            acc[0] += w;
            for (int o = 0; o < 16; ++o) acc[1 + o] += (pat == (uint32_t)o) ? w : 0.0;
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int v = 0; v < kRed; ++v) {
        double s = acc[v];
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
        if (lane == 0) sh[v][wv] = s;
    }
    __syncthreads();
    if (threadIdx.x < kRed) {
        double s = 0;
        for (int w = 0; w < kB / 64; ++w) s += sh[threadIdx.x][w];
        partial[(size_t)blockIdx.x * kRed + threadIdx.x] = s;
    }
}

// Keep the smallest relative decision margin of the shot (bits of a
// non-negative double).
__device__ __forceinline__ void keep_margin(uint64_t *marg, double m)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, m);
    if (b < *marg) *marg = b;
}

// Sum the partials in block order, draw, choose (first running sum above
// u*N, else the last candidate with weight), record measured bits and the
// decision margin. N is the Kraus channel's norm sum, or for a measurement
// the sum of its outcome probabilities in outcome order.
__global__ void k_decide(const double *partial, int nblocks, int cnt, uint64_t seed, uint64_t shot,
                         const DevOp *op, Cell *cell, uint64_t *mem, uint64_t *marg, double ro01,
                         double ro10)
{
    // sum the per-block partials: each thread a strided share, then a
    // fixed-order tree over the threads (the same order on every call)
    __shared__ double part[kRed][kB];
    __shared__ double red[kRed];
    const int t = threadIdx.x;
    for (int v = 0; v < kRed; ++v) {
        double s = 0;
        for (int b = t; b < nblocks; b += kB) s += partial[(size_t)b * kRed + v];
        part[v][t] = s;
    }
    __syncthreads();
    for (int w = kB / 2; w > 0; w >>= 1) {
        if (t < w)
            for (int v = 0; v < kRed; ++v) part[v][t] += part[v][t + w];
        __syncthreads();
    }
    if (t < kRed) red[t] = part[t][0];
    __syncthreads();
    if (t != 0) return;
    const double u = philox_u01(seed, shot, op->r, 0);
    double N = red[0];
    if (op->kind == DK_MEASURE) {
        N = 0;
        for (int t = 0; t < cnt; ++t) N += red[1 + t];
    }
    const double x = u * N;
    double run = 0, prev = 0;
    int o = -1, last = 0;
    for (int t = 0; t < cnt; ++t) {
        if (red[1 + t] > 0) last = t;
        prev = run;
        run += red[1 + t];
        if (x < run) { o = t; break; }
    }
    double mg = 0.0;  // the rounding fall-back is a tie
    if (o >= 0 && N > 0) {
        mg = __builtin_inf();
        if (o > 0) mg = fmin(mg, x - prev);
        if (o < cnt - 1) mg = fmin(mg, run - x);
        mg /= N;
    }
    keep_margin(marg, mg);
    if (o < 0) o = last;
    cell->outcome = o;
    cell->scale = 1.0 / sqrt(red[1 + o]);
    if (op->kind == DK_MEASURE && (op->flags & DF_RECORD)) {
        uint64_t m = *mem;
        for (int t = 0; t < op->nq; ++t) {
            uint64_t bit = (uint64_t)((o >> t) & 1);
            const double pf = bit ? ro10 : ro01;
            if (pf > 0 && philox_u01(seed, shot, op->r, 1u + t) < pf) bit ^= 1u;
            m = (m & ~(1ull << op->c[t])) | (bit << op->c[t]);
        }
        *mem = m;
    }
}

// Collapse onto the decided outcome and renormalise.
template <class R>
__global__ void k_collapse(typename V2<R>::T *st, uint64_t namps, const DevOp *op, const Cell *cell)
{
    const uint64_t i = (uint64_t)blockIdx.x * kB + threadIdx.x;
    if (i >= namps) return;
    uint32_t pat = 0;
    for (int t = 0; t < op->nq; ++t) pat |= (uint32_t)((i >> op->q[t]) & 1ull) << t;
    typename V2<R>::T v = st[i];
    if (pat == (uint32_t)cell->outcome) {
        v.x = (R)(v.x * cell->scale);
        v.y = (R)(v.y * cell->scale);
    } else {
        v.x = 0;
        v.y = 0;
    }
    st[i] = v;
}

// Reset: X on measured qubit t if the decided outcome has bit t set.
template <class R>
__global__ void k_reset_bit(typename V2<R>::T *st, uint64_t npairs, uint32_t q, int t, const Cell *cell)
{
    if (!((cell->outcome >> t) & 1)) return;
    const uint64_t p = (uint64_t)blockIdx.x * kB + threadIdx.x;
    if (p >= npairs) return;
    const uint64_t i0 = ins0(p, q), i1 = i0 | (1ull << q);
    const typename V2<R>::T a = st[i0];
    st[i0] = st[i1];
    st[i1] = a;
}

// Final measurement of all qubits: chunk sums (block b sums chunk b of
// kB amplitudes in a fixed tree), then one block samples.
template <class R>
__global__ void k_chunks(const typename V2<R>::T *st, uint64_t namps, double *chunk)
{
    __shared__ double sh[kB / 64];
    const uint64_t i = (uint64_t)blockIdx.x * kB + threadIdx.x;
    double s = 0;
    if (i < namps) {
        const typename V2<R>::T v = st[i];
        s = (double)v.x * v.x + (double)v.y * v.y;
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0;
        for (int w = 0; w < kB / 64; ++w) t += sh[w];
        chunk[blockIdx.x] = t;
    }
}

template <class R>
__global__ void k_sample(const typename V2<R>::T *st, uint64_t namps, const double *chunk,
                         uint64_t nchunks, int n, uint64_t seed, uint64_t shot, const DevOp *op,
                         uint64_t *mem, uint64_t *marg, double ro01, double ro10)
{
    if (threadIdx.x != 0) return;
    double N = 0;
    for (uint64_t b = 0; b < nchunks; ++b) N += chunk[b];
    const double x = philox_u01(seed, shot, op->r, 0) * N;
    // first chunk whose running sum passes x, then the first amplitude
    double run = 0;
    uint64_t b = 0, lastb = 0;
    for (; b < nchunks; ++b) {
        if (chunk[b] > 0) lastb = b;
        if (x < run + chunk[b]) break;
        run += chunk[b];
    }
    const bool fell_through = b == nchunks;
    if (fell_through) b = lastb;
    const uint64_t e0 = b * kB, e1 = (b + 1) * kB < namps ? (b + 1) * kB : namps;
    // margin: the chunk boundaries that chose chunk b, then the boundaries
    // of the chosen entry (the state's last entry has no upper boundary)
    double mg = __builtin_inf();
    if (b > 0) mg = fmin(mg, x - run);
    if (b + 1 < nchunks) mg = fmin(mg, run + chunk[b] - x);
    uint64_t idx = e0, lastnz = e0;
    bool found = false;
    for (uint64_t e = e0; e < e1; ++e) {
        const double w = (double)st[e].x * st[e].x + (double)st[e].y * st[e].y;
        if (w > 0) lastnz = e;
        const double before = run;
        run += w;
        if (!fell_through && x < run) {
            idx = e;
            found = true;
            if (e > e0) mg = fmin(mg, x - before);
            if (e + 1 < namps) mg = fmin(mg, run - x);
            break;
        }
    }
    if (!found) idx = lastnz;
    keep_margin(marg, found && N > 0 ? mg / N : 0.0);
    uint64_t m = *mem;
    for (int q = 0; q < n; ++q) {
        uint64_t bit = (idx >> q) & 1ull;
        const double pf = bit ? ro10 : ro01;
        if (pf > 0 && philox_u01(seed, shot, op->r, 1u + q) < pf) bit ^= 1u;
        m = (m & ~(1ull << op->c[q])) | (bit << op->c[q]);
    }
    *mem = m;
}

}  // namespace plain
}  // namespace svb

using namespace svb;
using namespace svb::plain;

// Run shots [0, n_shots) of the expanded program `ops` (device memory, list
// order) in plain form. hops: the same records on the host (for launch
// shapes). Returns the first launch error.
template <class R>
static hipError_t plain_run_t(const DevOp *ops, const DevOp *hops, int n_ops, const DevRule *rules,
                              const DevRule *hrules, const double *pool, int n, uint64_t n_shots,
                              uint64_t shot_base, uint64_t seed, void *state, uint64_t *memory,
                              uint64_t *margins, double *partial, int red_blocks, double *chunk,
                              void *cellp, double ro01, double ro10, hipStream_t st)
{
    using A = typename V2<R>::T;
    A *S = (A *)state;
    Cell *cell = (Cell *)cellp;
    const uint64_t namps = 1ull << n;
    const unsigned g1 = (unsigned)((namps + kB - 1) / kB);
    const unsigned g2 = (unsigned)((namps / 2 + kB - 1) / kB);
    const unsigned g4 = (unsigned)((namps / 4 + kB - 1) / kB);
    // reduction grid sized to the state (one block per 1024 amplitudes)
    red_blocks = (int)std::min<uint64_t>((uint64_t)red_blocks, std::max<uint64_t>(1, g4));
    for (uint64_t s = 0; s < n_shots; ++s) {
        const uint64_t shot = shot_base + s;
        uint64_t *mem = memory + s;
        uint64_t *marg = margins + s;
        hipLaunchKernelGGL(k_init<R>, dim3(g1), dim3(kB), 0, st, S, namps, mem, marg);
        for (int j = 0; j < n_ops; ++j) {
            const DevOp &h = hops[j];
            const DevOp *d = ops + j;
            switch (h.kind) {
            case DK_MAT1:
                hipLaunchKernelGGL(k_mat1<R>, dim3(g2), dim3(kB), 0, st, S, namps / 2, h.q[0],
                                   pool + h.mat, (const Cell *)nullptr, 0u);
                break;
            case DK_MATK:
                launch_dense<R>(S, n, h.nq, d, pool + h.mat, nullptr, 0u, st);
                break;
            case DK_CX:
            case DK_CZ:
            case DK_SWAP:
                hipLaunchKernelGGL(k_perm<R>, dim3(g4), dim3(kB), 0, st, S, namps / 4, h.q[0], h.q[1],
                                   h.kind == DK_CX ? 0 : h.kind == DK_CZ ? 1 : 2);
                break;
            case DK_PAULI: {
                const DevRule &hr = hrules[h.rule];
                hipLaunchKernelGGL(k_pauli_decide, dim3(1), dim3(1), 0, st, seed, shot, h.r,
                                   pool + hr.thr, (int)hr.n_terms, cell);
                hipLaunchKernelGGL(k_pauli_apply<R>, dim3(g1), dim3(kB), 0, st, S, namps,
                                   rules + h.rule, pool, d, (const Cell *)cell);
                break;
            }
            case DK_KRAUS: {
                const DevRule &hr = hrules[h.rule];
                hipLaunchKernelGGL(k_reduce<R>, dim3(red_blocks), dim3(kB), 0, st, (const A *)S, n, d,
                                   rules, pool, partial);
                hipLaunchKernelGGL(k_decide, dim3(1), dim3(kB), 0, st, (const double *)partial,
                                   red_blocks, (int)hr.n_terms, seed, shot, d, cell, mem, marg, ro01, ro10);
                const uint32_t dim = 1u << hr.nq;
                if (hr.nq == 1)
                    hipLaunchKernelGGL(k_mat1<R>, dim3(g2), dim3(kB), 0, st, S, namps / 2, h.q[0],
                                       pool + hr.mats, (const Cell *)cell, dim * dim * 2);
                else
                    launch_dense<R>(S, n, (int)hr.nq, d, pool + hr.mats, cell, dim * dim * 2, st);
                break;
            }
            case DK_MEASURE: {
                if (h.flags & DF_TERMINAL) {
                    hipLaunchKernelGGL(k_chunks<R>, dim3(g1), dim3(kB), 0, st, (const A *)S, namps,
                                       chunk);
                    hipLaunchKernelGGL(k_sample<R>, dim3(1), dim3(64), 0, st, (const A *)S, namps,
                                       (const double *)chunk, (uint64_t)g1, n, seed, shot, d, mem,
                                       marg, ro01, ro10);
                    break;
                }
                hipLaunchKernelGGL(k_reduce<R>, dim3(red_blocks), dim3(kB), 0, st, (const A *)S, n, d,
                                   rules, pool, partial);
                hipLaunchKernelGGL(k_decide, dim3(1), dim3(kB), 0, st, (const double *)partial,
                                   red_blocks, 1 << h.nq, seed, shot, d, cell, mem, marg, ro01, ro10);
                hipLaunchKernelGGL(k_collapse<R>, dim3(g1), dim3(kB), 0, st, S, namps, d,
                                   (const Cell *)cell);
                if (h.flags & DF_RESET)
                    for (int t = 0; t < h.nq; ++t)
                        hipLaunchKernelGGL(k_reset_bit<R>, dim3(g2), dim3(kB), 0, st, S, namps / 2,
                                           h.q[t], t, (const Cell *)cell);
                break;
            }
            default: break;
            }
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

extern "C" hipError_t svb_plain_run(int is_c128, const DevOp *ops, const DevOp *hops, int n_ops,
                                    const DevRule *rules, const DevRule *hrules, const double *pool,
                                    int n, uint64_t n_shots, uint64_t shot_base, uint64_t seed,
                                    void *state, uint64_t *memory, uint64_t *margins,
                                    double *partial, int red_blocks, double *chunk, void *cell,
                                    double ro01, double ro10, hipStream_t st)
{
    if (is_c128)
        return plain_run_t<double>(ops, hops, n_ops, rules, hrules, pool, n, n_shots, shot_base, seed,
                                   state, memory, margins, partial, red_blocks, chunk, cell, ro01,
                                   ro10, st);
    return plain_run_t<float>(ops, hops, n_ops, rules, hrules, pool, n, n_shots, shot_base, seed,
                              state, memory, margins, partial, red_blocks, chunk, cell, ro01, ro10,
                              st);
}
