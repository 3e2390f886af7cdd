/*
 * ckks_hip.h -- C ABI of the MI355X (gfx950) library for the key-switching
 * path of 32-bit-word RNS-CKKS, after Cheddar (arXiv 2407.13055).
 *
 * Operations (paper sections):
 *   NTT / INTT per limb set ............ Sec. 2.2 (Eq. 3 prime condition)
 *   BConv .............................. Sec. 2.2 Eq. 2, Sec. 2.3 Alg. 1
 *   KeySwitch (ModUp, KeyMult, ModDown)  Sec. 2.3
 *   HMult with relinearisation ......... Sec. 2.1 (HMult bullet, evk_mult)
 *   HRot with key switching ............ Sec. 2.1 (HRot bullet), Sec. 2.2 Eq. 4
 *   Rescale (single rescaling) ......... Sec. 2.1 "Rescaling", Sec. 3.1
 *
 * Conventions shared by every call
 *   - Residues are uint32, canonical in [0, q), standard (not Montgomery)
 *     form, limb-major: a polynomial over k primes is [k][N].
 *   - Evaluation (NTT) domain is bit-reversed:
 *       A[k] = sum_n a[n] psi^((2 brev(k) + 1) n)  (mod q),
 *     psi = the smallest g >= 2 with g^N = -1 (mod q).
 *   - Prime ids: 0..n_q-1 are the ciphertext primes q_i, n_q..n_q+n_p-1 the
 *     special primes p_k.  "Level" = number of active ciphertext primes
 *     (q_0..q_{level-1}).
 *   - Key-switching digits have width n_p (= alpha): at level l, digit j
 *     holds q_i for j*n_p <= i < min((j+1)*n_p, l); dnum = ceil(n_q/n_p).
 *   - A ciphertext at level l is [2][l][N]: b then a, NTT domain.  An input
 *     ciphertext may hold more limbs than the operation's level; its top
 *     limbs are ignored (the a half starts at row `level_in`).
 *   - An evaluation key is [dnum][2][n_q+n_p][N] (b then a), NTT domain,
 *     prepared for the top level and truncated to lower levels by row
 *     selection: evk_j.b = -a_j s + e_j + g_j s' with g_j = P on digit j's
 *     rows and 0 elsewhere; the relinearisation key has s' = s^2, the
 *     rotation key for rotation k has s' = phi_{5^k}(s).
 *
 * Memory and streams
 *   - Every data pointer is a DEVICE pointer on the device that was current
 *     at ckks_ctx_create, 16-byte aligned (CKKS_EALIGN otherwise).  The
 *     caller owns all buffers, including the workspace sized by
 *     ckks_workspace_size; the library never allocates or frees them.
 *   - `stream` is a hipStream_t (NULL = default stream).  Calls only
 *     enqueue work; buffers must stay alive until it completes.  Calls on
 *     one workspace must not overlap.
 *   - Outputs must not overlap inputs unless stated.
 *
 * Errors: every call returns CKKS_OK (0) or a negative code; nothing throws
 * or exits.  ckks_last_error() returns a thread-local description of the
 * last failure.  Argument errors are reported before anything is enqueued;
 * a failed kernel launch returns CKKS_EHIP.
 */
#ifndef CKKS_HIP_H
#define CKKS_HIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    CKKS_OK = 0,
    CKKS_EINVAL = -1,       /* bad argument (level, prime id, size, aliasing) */
    CKKS_EALIGN = -2,       /* a device pointer is not 16-byte aligned */
    CKKS_EWORKSPACE = -3,   /* workspace missing or smaller than required */
    CKKS_EHIP = -4,         /* HIP runtime error */
    CKKS_EUNSUPPORTED = -5  /* parameters outside what the kernels support */
};

/* Operation codes for ckks_workspace_size. */
enum {
    CKKS_OP_BCONV = 1,
    CKKS_OP_KEYSWITCH = 2,
    CKKS_OP_HMULT = 3,
    CKKS_OP_HROT = 4,
    CKKS_OP_RESCALE = 5,
    CKKS_OP_HROT_HOISTED = 6, /* n_in = number of rotations */
    CKKS_OP_HROT_SUM = 7,     /* ckks_hrot_sum_hoisted */
    CKKS_OP_RESCALE_RATIONAL = 8 /* n_in, n_out = input / output limbs */
};

/* Thread-local message describing the last failed call ("" if none). */
const char* ckks_last_error(void);

/* The `count` largest primes below 2^bits that are 1 (mod 2^(log_n+1)),
 * in descending order, written to the host array `out`.  A prime
 * generator for Eq. 3 (Sec. 6 names one among the library's utilities).
 * CKKS_EINVAL if fewer exist. */
int ckks_prime_chain(int bits, int log_n, int count, uint64_t* out);

typedef struct ckks_ctx ckks_ctx; /* opaque; immutable after creation */

typedef struct {
    uint32_t log_n;    /* ring degree N = 2^log_n, 12 <= log_n <= 16 */
    uint32_t n_q;      /* number of ciphertext primes */
    uint32_t n_p;      /* number of special primes (= digit width), <= 16 */
    const uint64_t* q; /* host array [n_q], each prime < 2^31, 1 mod 2N */
    const uint64_t* p; /* host array [n_p], same conditions */
} ckks_params;

/* Validate the primes (prime, < 2^31, 1 mod 2N, distinct, n_q + n_p <= 64)
 * and build the device tables (twiddles, base-conversion matrices, folded
 * constants) on the current device.  The primes are copied. */
int ckks_ctx_create(const ckks_params* params, ckks_ctx** out);

/* A context whose levels are windows of the ciphertext prime list, for the
 * 25-30 prime system with rational rescaling (Sec. 3.2) in the
 * inverted-terminal layout (Sec. 3.3): params->q is the whole list
 * [tau_{t-1} .. tau_0, q_0 .. q_{m-1}] (Q_max), and level w (w < n_win) holds
 * the primes q[win_start[w]] .. q[win_start[w] + win_len[w] - 1] (host
 * arrays, copied).  Every level uses the one key over P * Q_max: keys are
 * [dnum][2][n_q + n_p][N] with dnum = ceil(n_q / n_p), key digit k covering
 * list primes k n_p .. k n_p + n_p - 1; a window that starts inside a key
 * digit decomposes into the parts of the digits it meets (Sec. 2.3).
 *
 * On such a context every call's `level` argument is a window's limb count
 * (the windows must have distinct limb counts, which the 25-30 system's
 * levels do: each level adds modulus), limb i of a level-ℓ operand is
 * prime q[win_start + i], and inputs must be at exactly the operation level.
 * Plaintexts of PAdd / PMult hold the window's limbs; those of
 * ckks_hrot_sum_hoisted stay indexed by prime id over all n_q + n_p rows.
 * Rescaling is ckks_rescale_rational between windows, or merged into
 * HMult's ModDown by ckks_hmult_rescale (and its batched form, whose output
 * slots hold the window below max_level's limbs); ckks_rescale returns
 * CKKS_EUNSUPPORTED.  In batched calls every item names its window by limb
 * count and its slot holds that window's ciphertext in its first limbs; an
 * item whose count names no window (or, when rescaling, has no window below)
 * is skipped like an item outside the level range.
 * CKKS_EINVAL for an empty list, a window outside q, or two windows of the
 * same length. */
int ckks_ctx_create_windowed(const ckks_params* params, const int32_t* win_start, const int32_t* win_len, int n_win,
                             ckks_ctx** out);
void ckks_ctx_destroy(ckks_ctx* ctx);

/* Launch-shape knobs of a context (a tuner picks them by timing; results are
 * bit-identical for every setting; the defaults are what the tuner picks on
 * MI355X at N = 2^16), in the spirit of Sec. 4.2's fine-tuning
 * (how much work each thread takes, how NTT stages split into phases).  The
 * work-group shapes of the fused BConv + NTT column passes follow from the
 * digit width of Sec. 2.3's ModUp / ModDown; the column-tile order is a
 * property of the gfx950 launch (8 XCDs with private L2 caches). */
typedef struct {
    int32_t bconv_tpw_up;    /* ModUp BConv targets per work-group: 1, 2 or 4 (default 2) */
    int32_t bconv_tpw_down;  /* ModDown BConv targets per work-group: 1, 2 or 4 (default 2) */
    int32_t xcd_pair;        /* 1: the column tiles of one 128-byte line run on one XCD (default) */
    int32_t rows_per_thread; /* residues per thread of the stand-alone NTT row passes: 16 (default) or 4
                                (one wave per 256-point row, four radix-4 rounds) */
    int32_t col_threads;     /* threads per column-pass tile: 256 (16 columns, default), 512 (32 columns:
                                whole 128-byte rows; used where a column is >= 32 points, N >= 2^13) or
                                128 (twice the work-groups; used where N >= 2^15) */
    int32_t rows_per_thread_single; /* the same knob for launches of one operation (grid.z = 1): a single
                                       HMult has too few waves to hide memory latency with 16 residues per
                                       thread, a batched call has enough; default 4;
                                       0 = rows_per_thread */
    int32_t keymult_rows;    /* residues per thread of KeyMult (with its NTT and INTT row passes): 16 or
                                4 (default; one wave per row, digit products summed in 64 bits) */
    int32_t keymult_rows_single; /* the same for launches of one operation (default 4); 0 = keymult_rows */
    int32_t cols_per_thread;  /* residues per thread of key switching's column passes (INTT columns, BConv +
                                 NTT columns): 16 (col_threads tiles) or 4 (default; 256-thread tiles of
                                 1024 / 2^(log_n - 8) columns, radix-4 rounds) */
    int32_t cols_per_thread_single; /* the same for launches of one operation (default 4);
                                       0 = cols_per_thread */
} ckks_tuning;

/* Set the knobs and rebuild the context's launch plans.  Synchronizes the
 * device first; must not run concurrently with any other call on `ctx`.
 * Workspace sizes do not change.  CKKS_EINVAL for values out of range. */
int ckks_ctx_tune(ckks_ctx* ctx, const ckks_tuning* tuning);
/* Current knobs of `ctx`. */
int ckks_ctx_tuning(const ckks_ctx* ctx, ckks_tuning* out);

/* Bytes of workspace that `op` needs at `level` (ignored for BCONV, which
 * takes n_in / n_out; other ops ignore those two). */
int ckks_workspace_size(const ckks_ctx* ctx, int op, int level, int n_in, int n_out, size_t* bytes);

/* In-place forward NTT of n_limbs limbs (coefficients, natural order ->
 * evaluation, bit-reversed order); limb i of `data` is modulo prime
 * prime_ids[i] (host array). */
int ckks_ntt(const ckks_ctx* ctx, uint32_t* data, const int32_t* prime_ids, int n_limbs, void* stream);
/* In-place inverse NTT (exact inverse of ckks_ntt). */
int ckks_intt(const ckks_ctx* ctx, uint32_t* data, const int32_t* prime_ids, int n_limbs, void* stream);

/* Fast base conversion, coefficient domain (Eq. 2 with the centred
 * representative): for every target t,
 *   out_t = sum_s lift_s(in_s * [S_s^-1]_s) * S_s  (mod t),  S_s = prod(S)/s,
 * lift_s(v) = v if 2v < s else v - s.  in [n_in][N], out [n_out][N];
 * in_ids (distinct) / out_ids are host arrays of prime ids; n_in, n_out <= 64.
 * Workspace: ckks_workspace_size(CKKS_OP_BCONV, 0, n_in, n_out). */
int ckks_bconv(const ckks_ctx* ctx, const uint32_t* in, const int32_t* in_ids, int n_in, uint32_t* out,
               const int32_t* out_ids, int n_out, void* ws, size_t ws_bytes, void* stream);

/* Key switching of d [level][N] (NTT domain over q_0..q_{level-1}) with
 * evaluation key evk:  (out0, out1) = (ModDown(ks0), ModDown(ks1)),
 * ks_h = sum_j ModUp_j(d) * evk_j.h  over the rows q_0..q_{level-1},
 * p_0..p_{n_p-1}  (Sec. 2.3).  out0, out1: [level][N]. */
int ckks_keyswitch(const ckks_ctx* ctx, const uint32_t* d, int level, const uint32_t* evk, uint32_t* out0,
                   uint32_t* out1, void* ws, size_t ws_bytes, void* stream);

/* HMult with relinearisation (Sec. 2.1): for (b_a, a_a), (b_b, a_b) at
 * levels level_a, level_b >= level, out [2][level][N] =
 *   (b_a b_b + u0, b_a a_b + a_a b_b + u1),  (u0, u1) = KeySwitch(a_a a_b, rlk).
 * The scale of the result is the product of the input scales. */
int ckks_hmult(const ckks_ctx* ctx, const uint32_t* ct_a, int level_a, const uint32_t* ct_b, int level_b,
               const uint32_t* rlk, int level, uint32_t* out, void* ws, size_t ws_bytes, void* stream);

/* HMult with relinearisation followed by rescale (Sec. 2.1), level >= 2:
 * out [2][level-1][N] equals ckks_rescale(ckks_hmult(...)) bit for bit.
 * The rescale is folded into ModDown (one pass fewer per limb): the last
 * limb of the key-switched result is formed in coefficient form from
 * ModDown's own base conversion, and its NTT rides on ModDown's NTT by
 * linearity.  The scale of the result is (scale_a * scale_b) / q_{level-1}.
 * Workspace: ckks_workspace_size(CKKS_OP_HMULT, level).
 *
 * On a windowed context (ckks_ctx_create_windowed) the rescaling is
 * rational, to the window with the next smaller limb count L' (out
 * [2][L'][N]; CKKS_EINVAL at the lowest window), and ModDown is merged into
 * it (the merge of Sec. 5-6, extended to the 25-30 system): with x the
 * KeyMult sums plus P (d0, d1) over the window and P, D the window's primes
 * outside the window below and A the primes it adds,
 *   out = round(Q_A x / (P Q_D))  over the window below,
 * one rounding instead of ModDown's and the rescaling's; it differs from
 * ckks_hmult followed by ckks_rescale_rational by a few units per
 * coefficient.  The scale is (scale_a * scale_b) * Q_A / Q_D. */
int ckks_hmult_rescale(const ckks_ctx* ctx, const uint32_t* ct_a, int level_a, const uint32_t* ct_b, int level_b,
                       const uint32_t* rlk, int level, uint32_t* out, void* ws, size_t ws_bytes, void* stream);

/* HRot (Sec. 2.1; automorphism Eq. 4): rotates slots left by k using the
 * Galois element g = 5^(k mod N/2) mod 2N:
 *   out [2][level][N] = (phi_g(b) + u0, u1),  (u0, u1) = KeySwitch(phi_g(a), rk),
 * rk the rotation key for k (switches phi_g(s) -> s).  ct at level_in >= level. */
int ckks_hrot(const ckks_ctx* ctx, const uint32_t* ct, int level_in, int level, int k, const uint32_t* rk,
              uint32_t* out, void* ws, size_t ws_bytes, void* stream);

/* Rescale by the last prime (Sec. 2.1): ct [2][level][N] -> out
 * [2][level-1][N],  t = lift(INTT(c_{level-1})),
 * c'_i = (c_i - NTT([t]_{q_i})) * q_{level-1}^-1  (mod q_i)  (round to
 * nearest of X / q_{level-1}).  level >= 2; out must not overlap ct. */
int ckks_rescale(const ckks_ctx* ctx, const uint32_t* ct, int level, uint32_t* out, void* ws, size_t ws_bytes,
                 void* stream);

/* Rational rescaling (Sec. 3.2, 25-30 prime system; the sequence of
 * Sec. 5.1): a ciphertext over the primes in_ids (host array of n_in prime
 * ids of this context, q's and p's numbered 0..n_q+n_p-1) goes to the
 * primes out_ids, dividing by Q_D / Q_A for D = dropped and A = added
 * primes: out_o = (Q_A x_o - BConv_{D->o}([Q_A x]_D)) Q_D^-1 mod o (x_o = 0
 * for added o), the base conversion with the centred lift of Eq. 2, in the
 * evaluation domain (INTT of the dropped limbs, NTT of the conversion).  In
 * the inverted-terminal layout every level's primes are a contiguous window
 * of the list [tau_{T-1}..tau_0, q_0..q_{M-1}] given to the context as its
 * ciphertext primes.  ct: [2][n_in][N], out: [2][n_out][N] (limb o holds
 * out_ids[o]); at least one prime is dropped; out and ws must not overlap ct.
 * ws_bytes >= ckks_workspace_size(CKKS_OP_RESCALE_RATIONAL, 0, n_in, n_out). */
int ckks_rescale_rational(const ckks_ctx* ctx, const uint32_t* ct, int n_in, const int32_t* in_ids, int n_out,
                          const int32_t* out_ids, uint32_t* out, void* ws, size_t ws_bytes, void* stream);

/* ---- Ciphertexts with their level and scale (Sec. 2.1) ----
 * The calls above take raw residue buffers; these carry a ciphertext's
 * metadata the way Sec. 2.1 tracks it: HMult multiplies the scales,
 * rescaling divides by the dropped modulus (single rescaling: q_{level-1};
 * rational rescaling on a windowed context: Q_D / Q_A, the dropped over the
 * added primes of Sec. 3.2), HRot keeps it.  Each call validates and enqueues
 * exactly as the raw call it names (same buffers, same errors, same result
 * residues), then sets out->level and out->scale; out->data must point at
 * the caller's output buffer.  On error *out is left unchanged. */
typedef struct {
    uint32_t* data;  /* [2][level][N]: b then a, evaluation domain (device) */
    int32_t level;   /* limbs per half (number of active ciphertext primes) */
    double scale;    /* the encoding scale Delta of the message it holds */
} ckks_ct;
/* as ckks_hmult: out->level = level, out->scale = a->scale * b->scale */
int ckks_ct_hmult(const ckks_ctx* ctx, const ckks_ct* a, const ckks_ct* b, const uint32_t* rlk, int level,
                  ckks_ct* out, void* ws, size_t ws_bytes, void* stream);
/* as ckks_hmult_rescale: out->level = the level below, out->scale =
 * a->scale * b->scale / q_{level-1} (windowed context: * Q_A / Q_D) */
int ckks_ct_hmult_rescale(const ckks_ctx* ctx, const ckks_ct* a, const ckks_ct* b, const uint32_t* rlk, int level,
                          ckks_ct* out, void* ws, size_t ws_bytes, void* stream);
/* as ckks_rescale on in->data at in->level: out->level = in->level - 1,
 * out->scale = in->scale / q_{in->level - 1} */
int ckks_ct_rescale(const ckks_ctx* ctx, const ckks_ct* in, ckks_ct* out, void* ws, size_t ws_bytes, void* stream);
/* as ckks_hrot: out->level = level, out->scale = in->scale */
int ckks_ct_hrot(const ckks_ctx* ctx, const ckks_ct* in, int level, int k, const uint32_t* rk, ckks_ct* out, void* ws,
                 size_t ws_bytes, void* stream);

/* ---- Element-wise mechanisms and conjugation (Sec. 2.1) ----
 * Ciphertexts [2][level_x][N] (b then a), evaluation domain; the operation
 * uses their first `level` limbs.  Plaintexts pt: [pt_limbs][N] residues of
 * an encoded message in the evaluation domain (rows q_0..; level <= pt_limbs
 * <= n_q + n_p, so a plaintext prepared over all primes serves too).  `out`
 * [2][level][N] may be the first operand itself (in place, when that operand
 * is at `level`; for HAdd also the second); any other overlap is rejected.
 * No workspace; HBM-bound single launches. */
/* HAdd: out = ct_a + ct_b (component-wise). */
int ckks_hadd(const ckks_ctx* ctx, const uint32_t* ct_a, int level_a, const uint32_t* ct_b, int level_b, int level,
              uint32_t* out, void* stream);
/* PAdd: out = (b + pt, a). */
int ckks_padd(const ckks_ctx* ctx, const uint32_t* ct, int level_in, const uint32_t* pt, int pt_limbs, int level,
              uint32_t* out, void* stream);
/* PMult: out = (b * pt, a * pt) slot-wise (the scale multiplies; rescale after). */
int ckks_pmult(const ckks_ctx* ctx, const uint32_t* ct, int level_in, const uint32_t* pt, int pt_limbs, int level,
               uint32_t* out, void* stream);
/* HConj: conjugates every slot: the automorphism X -> X^(2N-1) (Eq. 4 with
 * g = 2N-1), then key switching with the conjugation key ck (layout of an
 * evk, switching phi_{2N-1}(s) -> s).  As ckks_hrot otherwise: out must not
 * overlap ct; ws_bytes >= ckks_workspace_size(CKKS_OP_HROT, level). */
int ckks_hconj(const ckks_ctx* ctx, const uint32_t* ct, int level_in, int level, const uint32_t* ck, uint32_t* out,
               void* ws, size_t ws_bytes, void* stream);

/* ---- Batched operations (many ciphertexts at uneven levels) ----
 * Items live in a DEVICE array the caller writes; launch sizes depend only
 * on (n, max_level), so a stream capture of one call (hipGraph) can be
 * replayed after rewriting the items and the inputs.  Inputs are n_src
 * slots at a fixed stride from the input base pointers; item i reads slot
 * items[i].src and writes output slot i, and uses workspace bytes
 * [i*W, (i+1)*W), W = ckks_workspace_size(op, max_level).  An item whose
 * level, key index or input slot is out of range is skipped (its output
 * slot is not written); nothing outside the given buffers is accessed.
 * A batched call needs every level up to max_level to run ModUp's base
 * conversion in one launch (at most 128 target rows, i.e. dnum*(level +
 * n_p) - level <= 128); otherwise it returns CKKS_EUNSUPPORTED and the
 * single-operation calls serve. */
typedef struct {
    int32_t level;    /* operation level of the item, <= max_level */
    int32_t key;      /* key index (HRot batches), else 0 */
    int32_t rot;      /* rotation k (HRot batches), else 0 */
    int32_t src;      /* input slot, 0 <= src < n_src */
} ckks_batch_item;

/* HMult + relinearisation + rescale of n pairs (item level >= 2, key 0):
 * a, b: [n_src][2][level_in][N]; out: [n][2][max_level-1][N] -- item i's result
 * has level_i - 1 valid rows in each half (the a half starts at row
 * max_level-1 of its slot).  Bit-identical per item to ckks_hmult_rescale.
 * ws_bytes >= n * ckks_workspace_size(CKKS_OP_HMULT, max_level). */
int ckks_hmult_rescale_batch(const ckks_ctx* ctx, int n, const uint32_t* a, const uint32_t* b, int n_src, int level_in,
                             const ckks_batch_item* items, int max_level, const uint32_t* rlk, uint32_t* out,
                             void* ws, size_t ws_bytes, void* stream);

/* HMult + relinearisation of n pairs without rescale (item level >= 1,
 * key 0): as ckks_hmult_rescale_batch but out: [n][2][max_level][N], item
 * i's result has level_i valid rows per half.  Bit-identical per item to
 * ckks_hmult.  ws_bytes >= n * ckks_workspace_size(CKKS_OP_HMULT, max_level). */
int ckks_hmult_batch(const ckks_ctx* ctx, int n, const uint32_t* a, const uint32_t* b, int n_src, int level_in,
                     const ckks_batch_item* items, int max_level, const uint32_t* rlk, uint32_t* out, void* ws,
                     size_t ws_bytes, void* stream);

/* HRot of n ciphertexts: ct: [n_src][2][level_in][N]; item i rotates by rot_i
 * with key keys + key_i * (dnum*2*(n_q+n_p)*N) (keys: [n_keys][dnum][2][n_q+n_p][N]);
 * out: [n][2][max_level][N], level_i valid rows per half.  Bit-identical
 * per item to ckks_hrot.  ws_bytes >= n * ckks_workspace_size(CKKS_OP_HROT, max_level). */
int ckks_hrot_batch(const ckks_ctx* ctx, int n, const uint32_t* ct, int n_src, int level_in,
                    const ckks_batch_item* items, int max_level, const uint32_t* keys, int n_keys, uint32_t* out,
                    void* ws, size_t ws_bytes, void* stream);

/* Hoisted HRot (hoisting the shared ModUp across rotations; key switching
 * is linear and the centred base conversion commutes with the
 * automorphism, Sec. 2.3): n_rot rotations of one ciphertext ct
 * [2][level_in][N] at `level`, sharing one ModUp of its a half.  Rotation i
 * uses items[i].rot and key keys + items[i].key * (dnum*2*(n_q+n_p)*N);
 * items[i].level must equal `level` (items that do not, or whose key index
 * is outside [0, n_keys), are skipped); items[i].src is not used.  outs: [n_rot][2][level][N], each
 * bit-identical to ckks_hrot with the same rotation and key.  Workspace:
 * ckks_workspace_size(CKKS_OP_HROT_HOISTED, level, n_rot, 0). */
int ckks_hrot_hoisted(const ckks_ctx* ctx, const uint32_t* ct, int level_in, int level, int n_rot,
                      const ckks_batch_item* items, const uint32_t* keys, int n_keys, uint32_t* outs, void* ws,
                      size_t ws_bytes, void* stream);

/* Sum of plaintext-weighted rotations, the inner sum of a linear transform
 * (Sec. 5 Par.4/Par.5, Eq. 5):  out = sum_i pt_i * HRot(ct, rot_i), computed
 * with one ModUp of a (hoisted), one KeyMult pass that gathers every
 * rotation's automorphism, weights it by pt_i and accumulates over Q_l u P,
 * and one ModDown.  Not bit-identical to the sum of separate HRot + PMult
 * results (one rounding of ModDown instead of n_rot); the same up to the
 * key-switching error.  ct: [2][level_in][N]; items: DEVICE array of n_rot
 * {level (= level), key, rot, src (unused)}; keys: [n_keys][dnum][2][n_q+n_p][N];
 * pts: [n_rot][n_q+n_p][N] evaluation-domain plaintexts over ALL primes (rows
 * q_0..q_{n_q-1}, p_0..; rows q_level.. unused); out: [2][level][N], must not
 * overlap ct or pts.  Items with another level or a key index outside
 * [0, n_keys) contribute nothing.
 * ws_bytes >= ckks_workspace_size(CKKS_OP_HROT_SUM, level, 0, 0). */
int ckks_hrot_sum_hoisted(const ckks_ctx* ctx, const uint32_t* ct, int level_in, int level, int n_rot,
                          const ckks_batch_item* items, const uint32_t* keys, int n_keys, const uint32_t* pts,
                          uint32_t* out, void* ws, size_t ws_bytes, void* stream);


/* Kernel timing, for benchmarks and tracing (no paper passage; changes no
 * result).  ckks_profile_start preallocates 2*max_launches hipEvents and
 * from then on brackets every kernel the library enqueues with two of them
 * (launches beyond max_launches are not recorded); ckks_profile_stop ends
 * recording.  ckks_profile_kernels waits for the recorded events and
 * aggregates them by kernel name; ckks_profile_kernel returns entry i
 * (name is a static string).  Not thread-safe: use on one thread while no
 * other call runs on the context. */
int ckks_profile_start(ckks_ctx* ctx, int max_launches);
int ckks_profile_stop(ckks_ctx* ctx);
int ckks_profile_kernels(ckks_ctx* ctx, int* n_kernels);
int ckks_profile_kernel(ckks_ctx* ctx, int i, const char** name, int* launches, double* total_ms);

/* ---- Allocation-free HMult + relinearisation + rescale ----
 * For callers that cannot allocate device memory or take a workspace
 * argument: code under stream capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, checks, launches and result residues as
 * ckks_hmult_rescale, without ws / ws_bytes: the key-switching workspace is
 * the library's own scratch array of CKKS_NOALLOC_SCRATCH_BYTES in device
 * memory, one per GPU, held from the first context created on that GPU until
 * the process ends.  The call allocates and frees nothing.  A level whose
 * workspace (ckks_workspace_size(CKKS_OP_HMULT, level)) exceeds the array is
 * refused with CKKS_EWORKSPACE.  Every call on one GPU uses that GPU's one
 * array: calls that overlap on a GPU (other streams, other contexts, other
 * host threads) race on it, so issue them on one stream.  Nothing in the
 * array needs to start at zero; it keeps the last call's intermediates. */
#define CKKS_NOALLOC_SCRATCH_BYTES (64u << 20)
int ckks_hmult_rescale_noalloc(const ckks_ctx* ctx, const uint32_t* ct_a, int level_a, const uint32_t* ct_b,
                               int level_b, const uint32_t* rlk, int level, uint32_t* out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* CKKS_HIP_H */
