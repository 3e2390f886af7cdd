/*
 * ckks_oracle.c -- plain, slow, obviously-correct CPU reference for the
 * 32-bit-word RNS-CKKS key-switching path of Cheddar (arXiv 2407.13055):
 * negacyclic NTT / INTT, base conversion (BConv), ModUp, KeyMult, ModDown,
 * automorphism, rescale, HMult and HRot.
 *
 * THIS IS TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  The GPU library shares no
 * code, header, table or constant generator with this file, and never calls
 * it.
 *
 * Arithmetic: every modulus is below 2^32, so a product of two residues is
 * below 2^64 and fits a uint64_t; every step below is exact modular
 * arithmetic in uint64_t, reduced with the % operator.  No Montgomery form,
 * no lazy ranges, no fusion: each function follows one definition.
 *
 * Conventions (the paper leaves these open; the reading taken is stated):
 *  - Prime condition q = 1 (mod 2N)  (Sec. 2.2, Eq. 3); every prime < 2^31
 *    (Sec. 3).
 *  - psi_q = the smallest g in [2, q) with g^N = -1 (mod q); it is a
 *    primitive 2N-th root of unity.
 *  - Evaluation (NTT) domain is stored in bit-reversed order:
 *        A[k] = sum_n a[n] * psi^((2*brev(k)+1)*n)  (mod q).
 *  - lift_q(v) = v if 2v < q else v - q  (centred representative, q odd).
 *  - BConv (Sec. 2.2, Eq. 2; Alg. 1): y_s = lift_s(x_s * [S_s^-1]_s) with
 *    S_s = prod(S)/s, out_t = sum_s y_s * S_s  (mod t).  The centred
 *    representative is the one the lazy-reduction text of Sec. 4.2 prepares.
 *  - Digits (hybrid key switching): digit width = number of special
 *    primes alpha; at level l (= number of active ciphertext primes) digit j
 *    holds q_i for j*alpha <= i < min((j+1)*alpha, l).
 *  - ModUp / KeyMult / MAC / automorphism / ModDown order of HRot (Sec. 2.3).
 *  - Rescale (Sec. 2.1, single rescaling): divide by the last prime,
 *    rounding to nearest through the centred lift.
 *
 * Threads: the loops over limbs carry OpenMP pragmas.  The default build
 * ignores them (one thread); a separate timing build with -fopenmp spreads
 * the limbs over the host cores.  Limbs are independent, so the results are
 * the same either way.
 *
 * Buffers are uint32_t, limb-major: [limbs][N]; a ciphertext is [2][l][N]
 * (b then a); an evaluation key is [dnum][2][n_q+n_p][N] (b then a), rows
 * q_0..q_{n_q-1}, p_0..p_{n_p-1}.  All residues canonical in [0, q).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAX_PRIMES 64

typedef struct {
    int32_t log_n;
    int32_t n_q;                      /* ciphertext primes q_0..q_{n_q-1}      */
    int32_t n_p;                      /* special primes; also the digit width  */
    int32_t reserved;
    uint64_t mod[ORC_MAX_PRIMES];     /* q_0..q_{n_q-1}, then p_0..p_{n_p-1}   */
} orc_params;

/* ------------------------------------------------------------------ */
/* scalar modular arithmetic (moduli < 2^32)                          */
/* ------------------------------------------------------------------ */

static uint64_t mod_mul(uint64_t a, uint64_t b, uint64_t m) { return (a % m) * (b % m) % m; }
static uint64_t mod_add(uint64_t a, uint64_t b, uint64_t m) { return (a % m + b % m) % m; }
static uint64_t mod_sub(uint64_t a, uint64_t b, uint64_t m) { return (a % m + m - b % m) % m; }

static uint64_t mod_pow(uint64_t a, uint64_t e, uint64_t m)
{
    uint64_t r = 1 % m;
    a %= m;
    while (e) {
        if (e & 1) r = mod_mul(r, a, m);
        a = mod_mul(a, a, m);
        e >>= 1;
    }
    return r;
}

/* inverse modulo a prime m (Fermat) */
static uint64_t mod_inv(uint64_t a, uint64_t m) { return mod_pow(a, m - 2, m); }

/* reduce a signed 64-bit integer into [0, m) */
static uint64_t mod_signed(int64_t v, uint64_t m)
{
    int64_t r = v % (int64_t)m;
    if (r < 0) r += (int64_t)m;
    return (uint64_t)r;
}

/* centred representative of v in [0, q) */
static int64_t lift(uint64_t v, uint64_t q) { return (2 * v < q) ? (int64_t)v : (int64_t)v - (int64_t)q; }

static uint32_t bit_reverse(uint32_t x, int bits)
{
    uint32_t r = 0;
    for (int i = 0; i < bits; i++) {
        r = (r << 1) | (x & 1);
        x >>= 1;
    }
    return r;
}

/* ------------------------------------------------------------------ */
/* primes and roots (Sec. 2.2 Eq. 3; Sec. 6 prime generator)           */
/* ------------------------------------------------------------------ */

/* Deterministic Miller-Rabin for n < 2^32 (bases 2..37 are more than
 * enough below 3.3e24). */
int orc_is_prime(uint64_t n)
{
    static const uint64_t bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    if (n < 2) return 0;
    for (int i = 0; i < 12; i++) {
        if (n == bases[i]) return 1;
        if (n % bases[i] == 0) return 0;
    }
    uint64_t d = n - 1;
    int r = 0;
    while ((d & 1) == 0) { d >>= 1; r++; }
    for (int i = 0; i < 12; i++) {
        uint64_t x = mod_pow(bases[i], d, n);
        if (x == 1 || x == n - 1) continue;
        int composite = 1;
        for (int k = 1; k < r; k++) {
            x = mod_mul(x, x, n);
            if (x == n - 1) { composite = 0; break; }
        }
        if (composite) return 0;
    }
    return 1;
}

/* The `count` largest primes p < 2^bits with p = 1 (mod 2N), in descending
 * order.  Returns how many were found. */
int orc_prime_chain(int bits, int log_n, int count, uint64_t *out)
{
    uint64_t step = 2ull << log_n;
    uint64_t top = 1ull << bits;
    uint64_t c = ((top - 2) / step) * step + 1; /* largest candidate < 2^bits */
    int found = 0;
    while (found < count && c > step) {
        if (orc_is_prime(c)) out[found++] = c;
        c -= step;
    }
    return found;
}

/* All primes p < bound with p = 1 (mod step), ascending; returns the total
 * count (writes at most max_out). */
int orc_primes_below(uint64_t bound, uint64_t step, uint64_t *out, int max_out)
{
    int found = 0;
    for (uint64_t c = step + 1; c < bound; c += step) {
        if (orc_is_prime(c)) {
            if (found < max_out) out[found] = c;
            found++;
        }
    }
    return found;
}

/* psi_q: smallest g >= 2 with g^N = -1 (mod q).  The search is remembered
 * per (q, log_n) (a per-thread table of recent answers): for some primes the
 * smallest such g is large, and every transform of a limb asks again. */
uint64_t orc_find_psi(uint64_t q, int log_n)
{
    static _Thread_local uint64_t memo_q[64], memo_psi[64];
    static _Thread_local int memo_logn[64], memo_next;
    for (int i = 0; i < 64; i++)
        if (memo_q[i] == q && memo_logn[i] == log_n) return memo_psi[i];
    uint64_t n = 1ull << log_n, psi = 0;
    for (uint64_t g = 2; g < q; g++)
        if (mod_pow(g, n, q) == q - 1) { psi = g; break; }
    memo_q[memo_next] = q, memo_logn[memo_next] = log_n, memo_psi[memo_next] = psi;
    memo_next = (memo_next + 1) % 64;
    return psi;
}

/* ------------------------------------------------------------------ */
/* negacyclic NTT, written from its definition                         */
/*   A[k] = a(psi^(2*brev(k)+1)) = sum_n (a[n] psi^n) * omega^(n*brev(k)) */
/* with omega = psi^2: twist by psi^n, a length-N cyclic DFT (textbook  */
/* iterative radix-2), then store entry k at position brev(k).          */
/* ------------------------------------------------------------------ */

/* cyclic DFT in place: X[k] = sum_n x[n] w^(n k), w of order N */
static void cyclic_dft(uint64_t *x, int log_n, uint64_t w, uint64_t q)
{
    uint32_t n = 1u << log_n;
    /* input permutation to bit-reversed order */
    for (uint32_t i = 0; i < n; i++) {
        uint32_t j = bit_reverse(i, log_n);
        if (i < j) { uint64_t t = x[i]; x[i] = x[j]; x[j] = t; }
    }
    /* butterflies: sub-DFTs of length len, combined with powers of w_len */
    for (uint32_t len = 2; len <= n; len <<= 1) {
        uint64_t w_len = mod_pow(w, n / len, q);
        for (uint32_t start = 0; start < n; start += len) {
            uint64_t wk = 1;
            for (uint32_t k = 0; k < len / 2; k++) {
                uint64_t u = x[start + k];
                uint64_t v = mod_mul(x[start + k + len / 2], wk, q);
                x[start + k] = mod_add(u, v, q);
                x[start + k + len / 2] = mod_sub(u, v, q);
                wk = mod_mul(wk, w_len, q);
            }
        }
    }
}

void orc_ntt_limb(uint32_t *a, uint64_t q, int log_n)
{
    uint32_t n = 1u << log_n;
    uint64_t psi = orc_find_psi(q, log_n);
    uint64_t *x = (uint64_t *)malloc(sizeof(uint64_t) * n);
    uint64_t pw = 1;
    for (uint32_t i = 0; i < n; i++) {          /* twist */
        x[i] = mod_mul(a[i], pw, q);
        pw = mod_mul(pw, psi, q);
    }
    cyclic_dft(x, log_n, mod_mul(psi, psi, q), q);
    for (uint32_t k = 0; k < n; k++)            /* bit-reversed storage */
        a[bit_reverse(k, log_n)] = (uint32_t)x[k];
    free(x);
}

void orc_intt_limb(uint32_t *a, uint64_t q, int log_n)
{
    uint32_t n = 1u << log_n;
    uint64_t psi = orc_find_psi(q, log_n);
    uint64_t psi_inv = mod_inv(psi, q);
    uint64_t n_inv = mod_inv(n, q);
    uint64_t *x = (uint64_t *)malloc(sizeof(uint64_t) * n);
    for (uint32_t k = 0; k < n; k++) x[k] = a[bit_reverse(k, log_n)];
    cyclic_dft(x, log_n, mod_mul(psi_inv, psi_inv, q), q);  /* inverse DFT up to 1/N */
    uint64_t pw = n_inv;
    for (uint32_t i = 0; i < n; i++) {          /* untwist and scale by 1/N */
        a[i] = (uint32_t)mod_mul(x[i], pw, q);
        pw = mod_mul(pw, psi_inv, q);
    }
    free(x);
}

void orc_ntt(uint32_t *a, const uint64_t *mods, int n_limbs, int log_n)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < n_limbs; i++) orc_ntt_limb(a + ((size_t)i << log_n), mods[i], log_n);
}

void orc_intt(uint32_t *a, const uint64_t *mods, int n_limbs, int log_n)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < n_limbs; i++) orc_intt_limb(a + ((size_t)i << log_n), mods[i], log_n);
}

/* ------------------------------------------------------------------ */
/* BConv (Eq. 2 with the centred lift), coefficient domain             */
/* ------------------------------------------------------------------ */

void orc_bconv(const uint32_t *in, const uint64_t *in_mods, int n_in,
               uint32_t *out, const uint64_t *out_mods, int n_out, int log_n)
{
    size_t n = (size_t)1 << log_n;
    int64_t *y = (int64_t *)malloc(sizeof(int64_t) * n * n_in);
    /* BConv const mult: y_s = lift(x_s * [S_s^-1]_s) */
#pragma omp parallel for schedule(dynamic, 1)
    for (int s = 0; s < n_in; s++) {
        uint64_t shat = 1;
        for (int r = 0; r < n_in; r++)
            if (r != s) shat = mod_mul(shat, in_mods[r], in_mods[s]);
        uint64_t shat_inv = mod_inv(shat, in_mods[s]);
        for (size_t c = 0; c < n; c++)
            y[s * n + c] = lift(mod_mul(in[s * n + c], shat_inv, in_mods[s]), in_mods[s]);
    }
    /* BConv matrix mult: out_t = sum_s y_s * [S_s]_t */
#pragma omp parallel for schedule(dynamic, 1)
    for (int t = 0; t < n_out; t++) {
        uint64_t m = out_mods[t];
        uint64_t *col = (uint64_t *)malloc(sizeof(uint64_t) * n_in);
        for (int s = 0; s < n_in; s++) {
            uint64_t shat = 1;
            for (int r = 0; r < n_in; r++)
                if (r != s) shat = mod_mul(shat, in_mods[r], m);
            col[s] = shat;
        }
        for (size_t c = 0; c < n; c++) {
            uint64_t acc = 0;
            for (int s = 0; s < n_in; s++)
                acc = mod_add(acc, mod_mul(mod_signed(y[s * n + c], m), col[s], m), m);
            out[t * n + c] = (uint32_t)acc;
        }
        free(col);
    }
    free(y);
}

/* ------------------------------------------------------------------ */
/* ModUp, KeyMult, ModDown, KeySwitch (Sec. 2.3)                       */
/* ------------------------------------------------------------------ */

static int digit_lo(const orc_params *P, int j) { return j * P->n_p; }
static int digit_hi(const orc_params *P, int j, int level)
{
    int hi = (j + 1) * P->n_p;
    return hi < level ? hi : level;
}
static int num_digits(const orc_params *P, int level) { return (level + P->n_p - 1) / P->n_p; }

/* ModUp_j(d): d [level][N] NTT domain over q_0..q_{level-1}; out
 * [level+n_p][N] NTT domain over q_0..q_{level-1}, p_0..p_{n_p-1}. */
void orc_modup(const orc_params *P, const uint32_t *d, int level, int j, uint32_t *out)
{
    int log_n = P->log_n;
    size_t n = (size_t)1 << log_n;
    int lo = digit_lo(P, j), hi = digit_hi(P, j, level);
    int n_in = hi - lo, n_out = level - n_in + P->n_p;
    uint64_t in_mods[ORC_MAX_PRIMES], out_mods[ORC_MAX_PRIMES];
    int out_row[ORC_MAX_PRIMES];
    uint32_t *c = (uint32_t *)malloc(sizeof(uint32_t) * n * n_in);
    uint32_t *e = (uint32_t *)malloc(sizeof(uint32_t) * n * n_out);
    for (int s = 0; s < n_in; s++) in_mods[s] = P->mod[lo + s];
    memcpy(c, d + (size_t)lo * n, sizeof(uint32_t) * n * n_in);
    orc_intt(c, in_mods, n_in, log_n);
    int t = 0;
    for (int i = 0; i < level; i++)
        if (i < lo || i >= hi) { out_mods[t] = P->mod[i]; out_row[t] = i; t++; }
    for (int k = 0; k < P->n_p; k++) { out_mods[t] = P->mod[P->n_q + k]; out_row[t] = level + k; t++; }
    orc_bconv(c, in_mods, n_in, e, out_mods, n_out, log_n);
    orc_ntt(e, out_mods, n_out, log_n);
    for (int i = lo; i < hi; i++) memcpy(out + (size_t)i * n, d + (size_t)i * n, sizeof(uint32_t) * n);
    for (t = 0; t < n_out; t++) memcpy(out + (size_t)out_row[t] * n, e + (size_t)t * n, sizeof(uint32_t) * n);
    free(c);
    free(e);
}

/* ModDown: x [level+n_p][N] NTT over q_0..q_{level-1}, p_0..; out [level][N]
 * out_i = (x_i - NTT(BConv_{P->Q}(INTT(x_P)))_i) * P^-1  (mod q_i). */
void orc_moddown(const orc_params *P, const uint32_t *x, int level, uint32_t *out)
{
    int log_n = P->log_n;
    size_t n = (size_t)1 << log_n;
    uint64_t p_mods[ORC_MAX_PRIMES], q_mods[ORC_MAX_PRIMES];
    for (int k = 0; k < P->n_p; k++) p_mods[k] = P->mod[P->n_q + k];
    for (int i = 0; i < level; i++) q_mods[i] = P->mod[i];
    uint32_t *c = (uint32_t *)malloc(sizeof(uint32_t) * n * P->n_p);
    uint32_t *conv = (uint32_t *)malloc(sizeof(uint32_t) * n * level);
    memcpy(c, x + (size_t)level * n, sizeof(uint32_t) * n * P->n_p);
    orc_intt(c, p_mods, P->n_p, log_n);
    orc_bconv(c, p_mods, P->n_p, conv, q_mods, level, log_n);
    orc_ntt(conv, q_mods, level, log_n);
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < level; i++) {
        uint64_t q = q_mods[i], pinv = 1;
        for (int k = 0; k < P->n_p; k++) pinv = mod_mul(pinv, p_mods[k], q);
        pinv = mod_inv(pinv, q);
        for (size_t m = 0; m < n; m++)
            out[i * n + m] = (uint32_t)mod_mul(mod_sub(x[i * n + m], conv[i * n + m], q), pinv, q);
    }
    free(c);
    free(conv);
}

/* KeyMult over the digits of d, then ModDown of both halves. */
void orc_keyswitch(const orc_params *P, const uint32_t *d, int level, const uint32_t *evk,
                   uint32_t *out0, uint32_t *out1)
{
    size_t n = (size_t)1 << P->log_n;
    int rows = level + P->n_p, key_rows = P->n_q + P->n_p;
    uint32_t *up = (uint32_t *)malloc(sizeof(uint32_t) * n * rows);
    uint32_t *ks0 = (uint32_t *)calloc(n * rows, sizeof(uint32_t));
    uint32_t *ks1 = (uint32_t *)calloc(n * rows, sizeof(uint32_t));
    for (int j = 0; j < num_digits(P, level); j++) {
        orc_modup(P, d, level, j, up);
        const uint32_t *kb = evk + (size_t)(2 * j) * key_rows * n;
        const uint32_t *ka = evk + (size_t)(2 * j + 1) * key_rows * n;
#pragma omp parallel for schedule(dynamic, 1)
        for (int r = 0; r < rows; r++) {
            int key_row = r < level ? r : P->n_q + (r - level);   /* truncated top-level key */
            uint64_t m = P->mod[key_row];
            for (size_t c = 0; c < n; c++) {
                uint64_t u = up[r * n + c];
                ks0[r * n + c] = (uint32_t)mod_add(ks0[r * n + c], mod_mul(u, kb[key_row * n + c], m), m);
                ks1[r * n + c] = (uint32_t)mod_add(ks1[r * n + c], mod_mul(u, ka[key_row * n + c], m), m);
            }
        }
    }
    orc_moddown(P, ks0, level, out0);
    orc_moddown(P, ks1, level, out1);
    free(up);
    free(ks0);
    free(ks1);
}

/* ------------------------------------------------------------------ */
/* rescale, HMult, automorphism, HRot                                  */
/* ------------------------------------------------------------------ */

/* One polynomial c [level][N] (NTT) -> out [level-1][N]:
 * t = lift(INTT(c_{l-1})); out_i = (c_i - NTT([t]_{q_i})) * q_{l-1}^-1. */
void orc_rescale_poly(const orc_params *P, const uint32_t *c, int level, uint32_t *out)
{
    int log_n = P->log_n;
    size_t n = (size_t)1 << log_n;
    uint64_t ql = P->mod[level - 1];
    uint32_t *last = (uint32_t *)malloc(sizeof(uint32_t) * n);
    memcpy(last, c + (size_t)(level - 1) * n, sizeof(uint32_t) * n);
    orc_intt_limb(last, ql, log_n);
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < level - 1; i++) {
        uint64_t q = P->mod[i];
        uint64_t qinv = mod_inv(ql % q, q);
        uint32_t *ti = (uint32_t *)malloc(sizeof(uint32_t) * n);
        for (size_t m = 0; m < n; m++) ti[m] = (uint32_t)mod_signed(lift(last[m], ql), q);
        orc_ntt_limb(ti, q, log_n);
        for (size_t m = 0; m < n; m++)
            out[i * n + m] = (uint32_t)mod_mul(mod_sub(c[i * n + m], ti[m], q), qinv, q);
        free(ti);
    }
    free(last);
}

/* ct [2][level][N] -> out [2][level-1][N] */
void orc_rescale(const orc_params *P, const uint32_t *ct, int level, uint32_t *out)
{
    size_t n = (size_t)1 << P->log_n;
    orc_rescale_poly(P, ct, level, out);
    orc_rescale_poly(P, ct + (size_t)level * n, level, out + (size_t)(level - 1) * n);
}

/* HMult with relinearisation (Sec. 2.1): inputs are [2][level_x][N] at their
 * own levels, used at `level` (top limbs ignored).  out [2][level][N]. */
void orc_hmult(const orc_params *P, const uint32_t *cta, int level_a, const uint32_t *ctb, int level_b,
               const uint32_t *rlk, int level, uint32_t *out)
{
    size_t n = (size_t)1 << P->log_n;
    if (level < 1) return;
    const uint32_t *ba = cta, *aa = cta + (size_t)level_a * n;
    const uint32_t *bb = ctb, *ab = ctb + (size_t)level_b * n;
    uint32_t *d2 = (uint32_t *)malloc(sizeof(uint32_t) * n * level);
    uint32_t *u0 = (uint32_t *)malloc(sizeof(uint32_t) * n * level);
    uint32_t *u1 = (uint32_t *)malloc(sizeof(uint32_t) * n * level);
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < level; i++) {
        uint64_t q = P->mod[i];
        for (size_t m = 0; m < n; m++) d2[i * n + m] = (uint32_t)mod_mul(aa[i * n + m], ab[i * n + m], q);
    }
    orc_keyswitch(P, d2, level, rlk, u0, u1);
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < level; i++) {
        uint64_t q = P->mod[i];
        for (size_t m = 0; m < n; m++) {
            size_t x = i * n + m;
            uint64_t d0 = mod_mul(ba[x], bb[x], q);
            uint64_t d1 = mod_add(mod_mul(ba[x], ab[x], q), mod_mul(aa[x], bb[x], q), q);
            out[x] = (uint32_t)mod_add(d0, u0[x], q);
            out[(size_t)level * n + x] = (uint32_t)mod_add(d1, u1[x], q);
        }
    }
    free(d2);
    free(u0);
    free(u1);
}

/* Automorphism X -> X^g (g odd) in the bit-reversed NTT domain (Eq. 4):
 * natural-order slot k takes natural-order slot k' with
 * 2k'+1 = g(2k+1) (mod 2N). */
void orc_automorph_ntt(const uint32_t *in, uint32_t *out, int n_limbs, int log_n, uint64_t g)
{
    uint64_t n = 1ull << log_n, two_n = 2 * n;
    for (int l = 0; l < n_limbs; l++) {
        const uint32_t *src = in + ((size_t)l << log_n);
        uint32_t *dst = out + ((size_t)l << log_n);
        for (uint64_t k = 0; k < n; k++) {
            uint64_t kp = ((g % two_n) * (2 * k + 1) % two_n - 1) / 2;
            dst[bit_reverse((uint32_t)k, log_n)] = src[bit_reverse((uint32_t)kp, log_n)];
        }
    }
}

/* Automorphism in the coefficient domain: a(X) -> a(X^g), X^N = -1. */
void orc_automorph_coef(const uint32_t *in, uint32_t *out, const uint64_t *mods, int n_limbs, int log_n, uint64_t g)
{
    uint64_t n = 1ull << log_n, two_n = 2 * n;
    for (int l = 0; l < n_limbs; l++) {
        const uint32_t *src = in + ((size_t)l << log_n);
        uint32_t *dst = out + ((size_t)l << log_n);
        for (uint64_t i = 0; i < n; i++) {
            uint64_t e = (i * (g % two_n)) % two_n;
            if (e < n) dst[e] = src[i];
            else dst[e - n] = (uint32_t)mod_sub(0, src[i], mods[l]);
        }
    }
}

/* HRot (Sec. 2.3): out = (phi_g(b) + u0, u1), (u0, u1) = KeySwitch(phi_g(a), rk).
 * ct [2][level_in][N] used at `level`; out [2][level][N]. */
void orc_hrot(const orc_params *P, const uint32_t *ct, int level_in, int level, uint64_t g,
              const uint32_t *rk, uint32_t *out)
{
    size_t n = (size_t)1 << P->log_n;
    uint32_t *pb = (uint32_t *)malloc(sizeof(uint32_t) * n * level);
    uint32_t *pa = (uint32_t *)malloc(sizeof(uint32_t) * n * level);
    uint32_t *u0 = (uint32_t *)malloc(sizeof(uint32_t) * n * level);
    orc_automorph_ntt(ct, pb, level, P->log_n, g);
    orc_automorph_ntt(ct + (size_t)level_in * n, pa, level, P->log_n, g);
    orc_keyswitch(P, pa, level, rk, u0, out + (size_t)level * n);
    for (int i = 0; i < level; i++)
        for (size_t m = 0; m < n; m++)
            out[i * n + m] = (uint32_t)mod_add(pb[i * n + m], u0[i * n + m], P->mod[i]);
    free(pb);
    free(pa);
    free(u0);
}

/* Hoisted HRot: one ModUp of a shared by n_rot rotations; for rotation r,
 * ks = sum_j phi_{g_r}(ModUp_j(a)) * rk_r,j, then ModDown and add phi(b).
 * outs [n_rot][2][level][N]; rks[r] points at rotation key r. */
void orc_hrot_hoisted(const orc_params *P, const uint32_t *ct, int level_in, int level, int n_rot,
                      const uint64_t *g, const uint32_t *const *rks, uint32_t *outs)
{
    size_t n = (size_t)1 << P->log_n;
    int rows = level + P->n_p, key_rows = P->n_q + P->n_p, beta = num_digits(P, level);
    uint64_t row_mods[ORC_MAX_PRIMES];
    for (int r = 0; r < rows; r++) row_mods[r] = r < level ? P->mod[r] : P->mod[P->n_q + r - level];
    uint32_t *up = (uint32_t *)malloc(sizeof(uint32_t) * n * rows * beta);
    uint32_t *rot = (uint32_t *)malloc(sizeof(uint32_t) * n * rows);
    uint32_t *ks0 = (uint32_t *)malloc(sizeof(uint32_t) * n * rows);
    uint32_t *ks1 = (uint32_t *)malloc(sizeof(uint32_t) * n * rows);
    uint32_t *pb = (uint32_t *)malloc(sizeof(uint32_t) * n * level);
    for (int j = 0; j < beta; j++) orc_modup(P, ct + (size_t)level_in * n, level, j, up + (size_t)j * rows * n);
    for (int r = 0; r < n_rot; r++) {
        uint32_t *out = outs + (size_t)r * 2 * level * n;
        memset(ks0, 0, sizeof(uint32_t) * n * rows);
        memset(ks1, 0, sizeof(uint32_t) * n * rows);
        for (int j = 0; j < beta; j++) {
            orc_automorph_ntt(up + (size_t)j * rows * n, rot, rows, P->log_n, g[r]);
            const uint32_t *kb = rks[r] + (size_t)(2 * j) * key_rows * n;
            const uint32_t *ka = rks[r] + (size_t)(2 * j + 1) * key_rows * n;
            for (int row = 0; row < rows; row++) {
                int key_row = row < level ? row : P->n_q + (row - level);
                uint64_t m = row_mods[row];
                for (size_t c = 0; c < n; c++) {
                    uint64_t u = rot[row * n + c];
                    ks0[row * n + c] = (uint32_t)mod_add(ks0[row * n + c], mod_mul(u, kb[key_row * n + c], m), m);
                    ks1[row * n + c] = (uint32_t)mod_add(ks1[row * n + c], mod_mul(u, ka[key_row * n + c], m), m);
                }
            }
        }
        orc_moddown(P, ks0, level, out);
        orc_moddown(P, ks1, level, out + (size_t)level * n);
        orc_automorph_ntt(ct, pb, level, P->log_n, g[r]);
        for (int i = 0; i < level; i++)
            for (size_t m = 0; m < n; m++)
                out[i * n + m] = (uint32_t)mod_add(pb[i * n + m], out[i * n + m], P->mod[i]);
    }
    free(up);
    free(rot);
    free(ks0);
    free(ks1);
    free(pb);
}

/* Sum of plaintext-weighted rotations with one ModUp and one ModDown
 * (Sec. 5 Par.4/Par.5, Eq. 5; the "double hoisting" of linear transforms):
 *   ModUp(a) once (digits, evaluation domain, rows Q_l u P);
 *   ks_c = sum_r pt_r * sum_j phi_r(ModUp_j(a)) * evk_r,j.c  over Q_l u P;
 *   out = (ModDown(ks_0) + sum_r pt_r * phi_r(b), ModDown(ks_1)).
 * pts[r]: [n_q + n_p][N] evaluation-domain plaintext over all primes (rows
 * q_0..q_{n_q-1}, p_0..); rows q_l..q_{n_q-1} are not used. */
void orc_hrot_sum_hoisted(const orc_params *P, const uint32_t *ct, int level_in, int level, int n_rot,
                          const uint64_t *g, const uint32_t *const *rks, const uint32_t *const *pts, uint32_t *out)
{
    size_t n = (size_t)1 << P->log_n;
    int rows = level + P->n_p, key_rows = P->n_q + P->n_p, beta = num_digits(P, level);
    uint64_t row_mods[ORC_MAX_PRIMES];
    for (int r = 0; r < rows; r++) row_mods[r] = r < level ? P->mod[r] : P->mod[P->n_q + r - level];
    uint32_t *up = (uint32_t *)malloc(sizeof(uint32_t) * n * rows * beta);
    uint32_t *rot = (uint32_t *)malloc(sizeof(uint32_t) * n * rows);
    uint32_t *ks0 = (uint32_t *)calloc(n * rows, sizeof(uint32_t));
    uint32_t *ks1 = (uint32_t *)calloc(n * rows, sizeof(uint32_t));
    uint32_t *pb = (uint32_t *)malloc(sizeof(uint32_t) * n * level);
    uint32_t *bsum = (uint32_t *)calloc(n * level, sizeof(uint32_t));
    for (int j = 0; j < beta; j++) orc_modup(P, ct + (size_t)level_in * n, level, j, up + (size_t)j * rows * n);
    for (int r = 0; r < n_rot; r++) {
        for (int j = 0; j < beta; j++) {
            orc_automorph_ntt(up + (size_t)j * rows * n, rot, rows, P->log_n, g[r]);
            const uint32_t *kb = rks[r] + (size_t)(2 * j) * key_rows * n;
            const uint32_t *ka = rks[r] + (size_t)(2 * j + 1) * key_rows * n;
            for (int row = 0; row < rows; row++) {
                int key_row = row < level ? row : P->n_q + (row - level);
                uint64_t m = row_mods[row];
                for (size_t c = 0; c < n; c++) {
                    uint64_t u = mod_mul(rot[row * n + c], pts[r][key_row * n + c], m);
                    ks0[row * n + c] = (uint32_t)mod_add(ks0[row * n + c], mod_mul(u, kb[key_row * n + c], m), m);
                    ks1[row * n + c] = (uint32_t)mod_add(ks1[row * n + c], mod_mul(u, ka[key_row * n + c], m), m);
                }
            }
        }
        orc_automorph_ntt(ct, pb, level, P->log_n, g[r]);
        for (int i = 0; i < level; i++)
            for (size_t c = 0; c < n; c++)
                bsum[i * n + c] = (uint32_t)mod_add(bsum[i * n + c], mod_mul(pb[i * n + c], pts[r][i * n + c], P->mod[i]),
                                                    P->mod[i]);
    }
    orc_moddown(P, ks0, level, out);
    orc_moddown(P, ks1, level, out + (size_t)level * n);
    for (int i = 0; i < level; i++)
        for (size_t c = 0; c < n; c++) out[i * n + c] = (uint32_t)mod_add(out[i * n + c], bsum[i * n + c], P->mod[i]);
    free(up);
    free(rot);
    free(ks0);
    free(ks1);
    free(pb);
    free(bsum);
}

/* ------------------------------------------------------------------ */
/* helpers for key generation / encryption in the test harness         */
/* ------------------------------------------------------------------ */

/* signed integer coefficients -> residues mod each prime (coefficient
 * domain); out [n_limbs][N] */
void orc_reduce_signed(const int64_t *coef, const uint64_t *mods, int n_limbs, int log_n, uint32_t *out)
{
    size_t n = (size_t)1 << log_n;
    for (int l = 0; l < n_limbs; l++)
        for (size_t c = 0; c < n; c++) out[l * n + c] = (uint32_t)mod_signed(coef[c], mods[l]);
}

/* Threads the limb loops use (timing build with -fopenmp); returns the
 * count in effect, 1 in the default build. */
int orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
