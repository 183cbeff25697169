/*
 * CPU oracle for applying a wiring diagram of controlled-NOT steps to a
 * 2^M-entry state vector (Burger, "New approaches to quantum computer
 * simulation in a classical supercomputer", quant-ph/0308158).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file: only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code, header, table or helper with
 * the GPU library.
 *
 * What is computed (Sec. 2(a), 2(b), 2(h), 2(i) Summary of Method):
 *   k2 = U_L ... U_1 k1, where every U_s is the symmetric 0/1 permutation
 *   matrix of one wiring-diagram step: a NOT on target address bit a(goto)
 *   that fires when every controlling bit a(from) is 1 (Sec. 2(b)-(g)).
 *   U_s has a 1 at (i, i with bit goto flipped) for every row i whose
 *   control bits are all 1, and a 1 on the diagonal elsewhere.
 *
 * Signed steps (oracle_apply_signed, oracle_sample_rows_signed) add a
 * second step kind, a controlled phase of -1, which reaches the signed
 * permutation matrices such as the paper's first example (Sec. 2(a)).
 *
 * Conventions (readings of the paper, each listed in the design notes):
 *   - Address bit b (0-based) is the paper's a(b+1); a(1) is the LSB
 *     (Sec. 2(b)).  Rows are counted top to bottom from 0 to 2^M - 1.
 *   - steps[0] is U_1 and acts first.
 *   - Several controls are AND-ed (Sec. 2(g) generalised); a step with no
 *     control is the unconditional NOT of Sec. 2(e).
 *   - Amplitudes are opaque words: 8 bytes (complex64) or 16 bytes
 *     (complex128).  They are only moved, never read as floating point, so
 *     every result is exact to the bit.
 *
 * Every entry point returns 0 on success and a negative value when an
 * argument is out of range (M outside [1, 40], element size not 8 or 16, a
 * target >= M, a control >= M, a target among its own controls).
 */
#include <stdint.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_MAX_M 40u

/* Validation of one step list against M (the paper is silent on a control
 * equal to the target or a bit beyond the address width; such steps are
 * rejected). */
static int check_args(uint32_t M, uint32_t elem_bytes, const uint32_t *target,
                      const uint64_t *cmask, uint64_t L)
{
    if (M < 1u || M > ORACLE_MAX_M) return -1;
    if (elem_bytes != 8u && elem_bytes != 16u) return -1;
    if (L > 0 && (target == NULL || cmask == NULL)) return -1;
    uint64_t all = (M == 64u) ? ~0ull : ((1ull << M) - 1ull);
    for (uint64_t s = 0; s < L; ++s) {
        if (target[s] >= M) return -2;
        if (cmask[s] & ~all) return -2;
        if ((cmask[s] >> target[s]) & 1ull) return -2;
    }
    return 0;
}

/* Swap two amplitude words as raw 64-bit integers (one or two per entry). */
static inline void swap_words(uint64_t *w, uint64_t a, uint64_t b, uint32_t nw)
{
    for (uint32_t q = 0; q < nw; ++q) {
        uint64_t t = w[a * nw + q];
        w[a * nw + q] = w[b * nw + q];
        w[b * nw + q] = t;
    }
}

/*
 * Plain step-by-step update (the state is recomputed after every step,
 * Sec. 2(h) first sentence; the plain accumulation alternative of the
 * Conclusions).  For step s with target bit t and control set C, every row
 * i with bit t clear and all bits of C set is interchanged with row
 * i + 2^t (Sec. 2(d): partner offset 2^(goto-1) in 1-based numbering).
 * nthreads > 1 splits the loop over i among threads; the pairs of one step
 * are disjoint (Sec. 2(i) Parallelism: the loop of a step may be broken into
 * parts that run at the same time).
 */
int oracle_apply(uint32_t M, uint32_t elem_bytes, void *buf,
                 const uint32_t *target, const uint64_t *cmask, uint64_t L,
                 int nthreads)
{
    int rc = check_args(M, elem_bytes, target, cmask, L);
    if (rc) return rc;
    if (L > 0 && buf == NULL) return -1;
    uint64_t *w = (uint64_t *)buf;
    const uint32_t nw = elem_bytes / 8u;
    const uint64_t n = 1ull << M;
    for (uint64_t s = 0; s < L; ++s) {
        const uint64_t T = 1ull << target[s];
        const uint64_t C = cmask[s];
        int64_t i;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1) if (nthreads > 1)
#endif
        for (i = 0; i < (int64_t)n; ++i) {
            uint64_t u = (uint64_t)i;
            if ((u & T) == 0 && (u & C) == C) swap_words(w, u, u | T, nw);
        }
    }
    (void)nthreads;
    return 0;
}

/*
 * Looping over the interchanged rows only (Sec. 2(b) end, Sec. 2(i) Summary third bullet):
 * only the rows that are interchanged are visited.  A pair exists for every
 * assignment of the bits that are neither the target nor a control; a
 * counter over those free bits is spread into their positions, the control
 * bits are set to 1 and the target bit is left 0, which names the lower row
 * of each interchanged pair.  No row whose controls are 0 is ever looked at.
 */
int oracle_apply_enum(uint32_t M, uint32_t elem_bytes, void *buf,
                      const uint32_t *target, const uint64_t *cmask,
                      uint64_t L, int nthreads)
{
    int rc = check_args(M, elem_bytes, target, cmask, L);
    if (rc) return rc;
    if (L > 0 && buf == NULL) return -1;
    uint64_t *w = (uint64_t *)buf;
    const uint32_t nw = elem_bytes / 8u;
    for (uint64_t s = 0; s < L; ++s) {
        const uint64_t T = 1ull << target[s];
        const uint64_t C = cmask[s];
        uint32_t freepos[64];
        uint32_t nfree = 0;
        for (uint32_t b = 0; b < M; ++b)
            if (!((T | C) >> b & 1ull)) freepos[nfree++] = b;
        const uint64_t npairs = 1ull << nfree;
        int64_t q;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1) if (nthreads > 1)
#endif
        for (q = 0; q < (int64_t)npairs; ++q) {
            uint64_t lo = C; /* controls at 1, target at 0 */
            for (uint32_t f = 0; f < nfree; ++f)
                if (((uint64_t)q >> f) & 1ull) lo |= 1ull << freepos[f];
            swap_words(w, lo, lo | T, nw);
        }
    }
    (void)nthreads;
    return 0;
}

/*
 * Row array of one step (Sec. 2(b): y(i) holds the column of the single 1
 * in row i).  Because the step matrix is symmetric (Sec. 2(a)), the column
 * of row i is the row it is paired with: i with the target bit flipped
 * when every control bit of i is 1, else i itself.
 */
static inline uint64_t step_column(uint64_t i, uint64_t T, uint64_t C)
{
    return ((i & C) == C) ? (i ^ T) : i;
}

/*
 * The paper's sparse-matrix algorithm (Sec. 2(h), 2(i) Summary of Method):
 * start from the identity x(i) = i; for each step in the order given, build
 * the step's row array y and form the product x(i) <- y(x(i)); y returns to
 * the identity before the next step.  After the steps (S_1, ..., S_n) have
 * been folded in this order, x is the row array of the product
 * U_{S_1} U_{S_2} ... U_{S_n}, so x(i) is the column of the 1 in row i.
 * (The printed Fig. 2 intermediate x = (4,3,1,2) is exactly this product.)
 * x must hold 2^M entries.
 */
int oracle_rowmap(uint32_t M, const uint32_t *target, const uint64_t *cmask,
                  uint64_t L, uint64_t *x)
{
    int rc = check_args(M, 8u, target, cmask, L);
    if (rc) return rc;
    if (x == NULL) return -1;
    const uint64_t n = 1ull << M;
    for (uint64_t i = 0; i < n; ++i) x[i] = i;
    for (uint64_t s = 0; s < L; ++s) {
        const uint64_t T = 1ull << target[s];
        const uint64_t C = cmask[s];
        for (uint64_t i = 0; i < n; ++i) x[i] = step_column(x[i], T, C);
    }
    return 0;
}

/*
 * Column of the 1 in row i of U_L ... U_1 (the row array x(i) of the whole
 * wiring diagram for one row, Sec. 2(h)): following row i through the
 * product from the left, U_L sends it to y_L(i), then U_{L-1} to
 * y_{L-1}(y_L(i)), down to U_1.  The output entry is then k2(i) = k1(x(i))
 * (Sec. 2(b) end; Summary last bullet).  Used for sampled rows of states too
 * large for the plain loop.
 */
uint64_t oracle_source_index(uint32_t M, const uint32_t *target,
                             const uint64_t *cmask, uint64_t L, uint64_t i)
{
    (void)M;
    uint64_t x = i;
    for (uint64_t s = L; s-- > 0;)
        x = step_column(x, 1ull << target[s], cmask[s]);
    return x;
}

/*
 * k2 at sampled rows: out[r] = k1(x(idx[r])) for r < nsample (Sec. 2(b):
 * k2(i) = k1(x(i))).  k1 holds 2^M entries of elem_bytes each; out holds
 * nsample entries.
 */
int oracle_sample_rows(uint32_t M, uint32_t elem_bytes, const void *k1,
                       const uint32_t *target, const uint64_t *cmask,
                       uint64_t L, const uint64_t *idx, uint64_t nsample,
                       void *out, int nthreads)
{
    int rc = check_args(M, elem_bytes, target, cmask, L);
    if (rc) return rc;
    if (nsample > 0 && (k1 == NULL || idx == NULL || out == NULL)) return -1;
    const uint64_t n = 1ull << M;
    for (uint64_t r = 0; r < nsample; ++r)
        if (idx[r] >= n) return -3;
    const uint32_t nw = elem_bytes / 8u;
    const uint64_t *src = (const uint64_t *)k1;
    uint64_t *dst = (uint64_t *)out;
    int64_t r;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1) if (nthreads > 1)
#endif
    for (r = 0; r < (int64_t)nsample; ++r) {
        uint64_t x = oracle_source_index(M, target, cmask, L, idx[r]);
        for (uint32_t q = 0; q < nw; ++q) dst[(uint64_t)r * nw + q] = src[x * nw + q];
    }
    (void)nthreads;
    return 0;
}

/*
 * Input calculated from a Kronecker product of M qubit pairs (Appendix 1):
 * k1 = q_M (x) q_{M-1} (x) ... (x) q_1, so entry i is the product of
 * q_b(bit b-1 of i) over b = 1..M; e.g. k1(5) = q3(1) q2(0) q1(1).
 * The product is formed in the order printed there, from q_M down to q_1,
 * in the precision of the entries (float for elem_bytes 8, double for 16),
 * each complex product as (ac - bd) + (ad + bc)i with every operation
 * rounded separately (this file is compiled as ISO C, without contraction
 * of multiply-adds).  qubits holds q_b(v) at index 2(b-1) + v as
 * interleaved (re, im) pairs; out holds 2^M entries.
 */
int oracle_product_state(uint32_t M, uint32_t elem_bytes, const void *qubits, void *out)
{
    if (M < 1u || M > 30u) return -1;
    if (elem_bytes != 8u && elem_bytes != 16u) return -1;
    if (qubits == NULL || out == NULL) return -1;
    const uint64_t n = 1ull << M;
    if (elem_bytes == 8u) {
        const float *q = (const float *)qubits;
        float *o = (float *)out;
        for (uint64_t i = 0; i < n; ++i) {
            uint32_t b = M;                 /* qubit q_b, address bit b-1 */
            uint64_t v = (i >> (b - 1)) & 1u;
            float re = q[2 * (2 * (b - 1) + v)], im = q[2 * (2 * (b - 1) + v) + 1];
            for (b = M - 1; b >= 1; --b) {
                v = (i >> (b - 1)) & 1u;
                const float c = q[2 * (2 * (b - 1) + v)], d = q[2 * (2 * (b - 1) + v) + 1];
                const float ac = re * c, bd = im * d, ad = re * d, bc = im * c;
                re = ac - bd;
                im = ad + bc;
            }
            o[2 * i] = re;
            o[2 * i + 1] = im;
        }
    } else {
        const double *q = (const double *)qubits;
        double *o = (double *)out;
        for (uint64_t i = 0; i < n; ++i) {
            uint32_t b = M;
            uint64_t v = (i >> (b - 1)) & 1u;
            double re = q[2 * (2 * (b - 1) + v)], im = q[2 * (2 * (b - 1) + v) + 1];
            for (b = M - 1; b >= 1; --b) {
                v = (i >> (b - 1)) & 1u;
                const double c = q[2 * (2 * (b - 1) + v)], d = q[2 * (2 * (b - 1) + v) + 1];
                const double ac = re * c, bd = im * d, ad = re * d, bc = im * c;
                re = ac - bd;
                im = ad + bc;
            }
            o[2 * i] = re;
            o[2 * i + 1] = im;
        }
    }
    return 0;
}

/* One entry k1(i) of the same product (for rows of states too large to
 * form whole); out receives one entry of elem_bytes. */
int oracle_product_entry(uint32_t M, uint32_t elem_bytes, const void *qubits, uint64_t i, void *out)
{
    if (M < 1u || M > 40u || qubits == NULL || out == NULL) return -1;
    if (elem_bytes == 8u) {
        const float *q = (const float *)qubits;
        uint32_t b = M;
        uint64_t v = (i >> (b - 1)) & 1u;
        float re = q[2 * (2 * (b - 1) + v)], im = q[2 * (2 * (b - 1) + v) + 1];
        for (b = M - 1; b >= 1; --b) {
            v = (i >> (b - 1)) & 1u;
            const float c = q[2 * (2 * (b - 1) + v)], d = q[2 * (2 * (b - 1) + v) + 1];
            const float ac = re * c, bd = im * d, ad = re * d, bc = im * c;
            re = ac - bd;
            im = ad + bc;
        }
        ((float *)out)[0] = re;
        ((float *)out)[1] = im;
        return 0;
    }
    if (elem_bytes == 16u) {
        const double *q = (const double *)qubits;
        uint32_t b = M;
        uint64_t v = (i >> (b - 1)) & 1u;
        double re = q[2 * (2 * (b - 1) + v)], im = q[2 * (2 * (b - 1) + v) + 1];
        for (b = M - 1; b >= 1; --b) {
            v = (i >> (b - 1)) & 1u;
            const double c = q[2 * (2 * (b - 1) + v)], d = q[2 * (2 * (b - 1) + v) + 1];
            const double ac = re * c, bd = im * d, ad = re * d, bc = im * c;
            re = ac - bd;
            im = ad + bc;
        }
        ((double *)out)[0] = re;
        ((double *)out)[1] = im;
        return 0;
    }
    return -1;
}

/*
 * Signed steps (Sec. 2(a)).  The wiring-diagram class has only 0/1 step
 * matrices; the paper's first example of a unitary matrix, however, is a
 * permutation with one entry -1, which that class cannot reach.  A second
 * kind of step closes the gap: kind[s] = 1 is a controlled phase of -1,
 * the diagonal matrix with -1 in every row i whose bits t and C are all 1
 * and +1 elsewhere (symmetric, its own inverse, like every NOT step).
 * kind[s] = 0 is the controlled NOT above.  Products of both kinds are the
 * signed permutations reachable from controlled NOTs.
 *
 * Negating an entry negates its real and imaginary parts; IEEE 754
 * negation is the sign-bit flip, exact for every value (zeros, infinities
 * and NaN payloads included), so entries stay opaque words: bit 63 of each
 * 8-byte word for complex128, bits 31 and 63 of the one word for complex64.
 */
static int check_kinds(const uint8_t *kind, uint64_t L)
{
    if (L > 0 && kind == NULL) return -1;
    for (uint64_t s = 0; s < L; ++s)
        if (kind[s] > 1u) return -2;
    return 0;
}

static inline void negate_entry(uint64_t *w, uint64_t i, uint32_t nw)
{
    if (nw == 1u) {
        w[i] ^= (1ull << 31) | (1ull << 63);
    } else {
        w[2 * i] ^= 1ull << 63;
        w[2 * i + 1] ^= 1ull << 63;
    }
}

/* Plain loop over every row for every step, as oracle_apply, with phase
 * steps negating the rows whose bits t and C are all 1. */
int oracle_apply_signed(uint32_t M, uint32_t elem_bytes, void *buf,
                        const uint32_t *target, const uint64_t *cmask,
                        const uint8_t *kind, uint64_t L, int nthreads)
{
    int rc = check_args(M, elem_bytes, target, cmask, L);
    if (rc) return rc;
    if ((rc = check_kinds(kind, L))) return rc;
    if (L > 0 && buf == NULL) return -1;
    uint64_t *w = (uint64_t *)buf;
    const uint32_t nw = elem_bytes / 8u;
    const uint64_t n = 1ull << M;
    for (uint64_t s = 0; s < L; ++s) {
        const uint64_t T = 1ull << target[s];
        const uint64_t C = cmask[s];
        const int phase = kind[s] == 1u;
        int64_t i;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1) if (nthreads > 1)
#endif
        for (i = 0; i < (int64_t)n; ++i) {
            uint64_t u = (uint64_t)i;
            if (phase) {
                if ((u & (C | T)) == (C | T)) negate_entry(w, u, nw);
            } else if ((u & T) == 0 && (u & C) == C) {
                swap_words(w, u, u | T, nw);
            }
        }
    }
    (void)nthreads;
    return 0;
}

/*
 * Column x(i) and sign of row i of the signed product U_L ... U_1 (see
 * below): *neg receives 1 when the entry is -1.  Returns x(i).
 */
uint64_t oracle_source_index_signed(uint32_t M, const uint32_t *target, const uint64_t *cmask,
                                    const uint8_t *kind, uint64_t L, uint64_t i, int *neg)
{
    (void)M;
    uint64_t x = i;
    int n = 0;
    for (uint64_t s = L; s-- > 0;) {
        const uint64_t T = 1ull << target[s];
        if (kind[s] == 1u) {
            if ((x & (cmask[s] | T)) == (cmask[s] | T)) n ^= 1;
        } else {
            x = step_column(x, T, cmask[s]);
        }
    }
    if (neg) *neg = n;
    return x;
}

/*
 * k2 at sampled rows for signed steps.  Row i of U_L ... U_1 has its one
 * nonzero entry in column x(i) with sign sigma(i): following row i through
 * the product from the left, a NOT step U_s moves it to row y_s(i), and a
 * phase step multiplies it by U_s's diagonal entry in the row it is in at
 * that point.  out[r] = sigma(idx[r]) k1(x(idx[r])).
 */
int oracle_sample_rows_signed(uint32_t M, uint32_t elem_bytes, const void *k1,
                              const uint32_t *target, const uint64_t *cmask,
                              const uint8_t *kind, uint64_t L, const uint64_t *idx,
                              uint64_t nsample, void *out, int nthreads)
{
    int rc = check_args(M, elem_bytes, target, cmask, L);
    if (rc) return rc;
    if ((rc = check_kinds(kind, L))) return rc;
    if (nsample > 0 && (k1 == NULL || idx == NULL || out == NULL)) return -1;
    const uint64_t n = 1ull << M;
    for (uint64_t r = 0; r < nsample; ++r)
        if (idx[r] >= n) return -3;
    const uint32_t nw = elem_bytes / 8u;
    const uint64_t *src = (const uint64_t *)k1;
    uint64_t *dst = (uint64_t *)out;
    int64_t r;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1) if (nthreads > 1)
#endif
    for (r = 0; r < (int64_t)nsample; ++r) {
        uint64_t x = idx[r];
        int neg = 0;
        for (uint64_t s = L; s-- > 0;) {
            const uint64_t T = 1ull << target[s];
            if (kind[s] == 1u) {
                if ((x & (cmask[s] | T)) == (cmask[s] | T)) neg ^= 1;
            } else {
                x = step_column(x, T, cmask[s]);
            }
        }
        for (uint32_t q = 0; q < nw; ++q) dst[(uint64_t)r * nw + q] = src[x * nw + q];
        if (neg) negate_entry(dst, (uint64_t)r, nw);
    }
    (void)nthreads;
    return 0;
}

/* Number of threads an OpenMP region would use (1 without OpenMP). */
int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
