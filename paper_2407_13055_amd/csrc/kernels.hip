// HIP kernels and launch sequences of the key-switching path (gfx950):
// ModUp -> KeyMult -> MAC -> automorphism -> ModDown (Sec. 2.3), rescale
// (Sec. 2.1), and the stand-alone NTT / BConv calls.
//
// Fusion (Sec. 5): the tensor product, the automorphism gather and the BConv
// constant multiplication ride on the INTT passes (Seq.1); the BConv matrix
// multiplication feeds the NTT column pass directly; KeyMult over all digits
// is one output-stationary kernel that also runs the NTT row pass, adds the
// HMult d0/d1 (or HRot phi(b)) term pre-multiplied by P so that ModDown
// returns it unchanged, and starts ModDown's INTT on the P rows (Par.1); the
// last NTT row pass of ModDown / rescale subtracts and scales in its
// epilogue (Seq.3).  Montgomery factors 2^-32 are folded into constants
// (Seq.2) so no pass converts in or out of Montgomery form.
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <vector>

#include "internal.h"
#include "ntt_core.h"

namespace ckks {

thread_local KtEvents* g_kt = nullptr;

// ---------------------------------------------------------------------------
// loaders
// ---------------------------------------------------------------------------
__device__ __forceinline__ void load16_u32(const uint32_t* p, uint32_t (&x)[16])
{
    const uint4* v = reinterpret_cast<const uint4*>(p);
#pragma unroll
    for (int i = 0; i < 4; i++) {
        uint4 t = v[i];
        x[4 * i] = t.x, x[4 * i + 1] = t.y, x[4 * i + 2] = t.z, x[4 * i + 3] = t.w;
    }
}

__device__ __forceinline__ void store16_u32(uint32_t* p, const uint32_t (&x)[16])
{
    uint4* v = reinterpret_cast<uint4*>(p);
#pragma unroll
    for (int i = 0; i < 4; i++) v[i] = make_uint4(x[4 * i], x[4 * i + 1], x[4 * i + 2], x[4 * i + 3]);
}

// E contiguous residues (E a multiple of 4, p 16-byte aligned)
template <int E>
__device__ __forceinline__ void loadv_u32(const uint32_t* p, uint32_t (&x)[E])
{
    const uint4* v = reinterpret_cast<const uint4*>(p);
#pragma unroll
    for (int i = 0; i < E / 4; i++) {
        uint4 t = v[i];
        x[4 * i] = t.x, x[4 * i + 1] = t.y, x[4 * i + 2] = t.z, x[4 * i + 3] = t.w;
    }
}
template <int E>
__device__ __forceinline__ void storev_u32(uint32_t* p, const uint32_t (&x)[E])
{
    uint4* v = reinterpret_cast<uint4*>(p);
#pragma unroll
    for (int i = 0; i < E / 4; i++) v[i] = make_uint4(x[4 * i], x[4 * i + 1], x[4 * i + 2], x[4 * i + 3]);
}

// Galois element 5^(k mod N/2) mod 2N of a rotation by k slots (Sec. 2.2 Eq. 4)
__device__ __forceinline__ uint32_t galois_of(int k, int log_n)
{
    const uint32_t half = 1u << (log_n - 1), mask = (2u << log_n) - 1u;
    uint32_t e = (uint32_t)(((k % (int)half) + (int)half) % (int)half), g = 1, b = 5;
    for (; e; e >>= 1, b = (b * b) & mask)
        if (e & 1) g = (g * b) & mask;
    return g;
}

// bit-reversed position of the automorphism's source (Eq. 4, X -> X^g):
// natural slot k takes natural slot k' with 2k'+1 = g(2k+1) mod 2N.
__device__ __forceinline__ int aut_src(int pos, uint32_t g, int log_n)
{
    const uint32_t k = __brev((uint32_t)pos) >> (32 - log_n);
    const uint32_t kp = (((g * (2u * k + 1u)) & ((2u << log_n) - 1u)) - 1u) >> 1;
    return (int)(__brev(kp) >> (32 - log_n));
}

// Every loader / storer carries, per pointer, the residue step between
// consecutive items of a batched launch (0 for a single operation); at(i)
// returns the copy for item i.
struct LdPlain {
    static constexpr bool kTileThread = false;
    const uint32_t* base;
    int log_n;
    size_t step = 0;
    __device__ LdPlain at(int i) const
    {
        LdPlain r = *this;
        r.base += (size_t)i * step;
        return r;
    }
    __device__ uint32_t load(const LaunchMap& M, int l, int j, PrimeC) const
    {
        return base[((size_t)M.in_off[l] << log_n) + j];
    }
    __device__ void load16(const LaunchMap& M, int l, int j, PrimeC, uint32_t (&x)[16]) const
    {
        load16_u32(base + ((size_t)M.in_off[l] << log_n) + j, x);
    }
    template <int E>
    __device__ void loadv(const LaunchMap& M, int l, int j, PrimeC, uint32_t (&x)[E]) const
    {
        loadv_u32<E>(base + ((size_t)M.in_off[l] << log_n) + j, x);
    }
};

// the digit's own rows: a_a*a_b*2^-32 (HMult), d (KeySwitch), phi_g(a) (HRot)
template <Own OWN>
struct LdOwn {
    static constexpr bool kTileThread = false;
    const uint32_t* a0;
    const uint32_t* a1;
    uint32_t galois;
    int log_n;
    size_t step0 = 0, step1 = 0;
    const BatchItem* items = nullptr;  // batched HRot: Galois element per item
    __device__ LdOwn at(int i) const
    {
        LdOwn r = *this;
        const size_t src = items ? (size_t)items[i].src : (size_t)i;  // input slot of item i
        r.a0 += src * step0;
        if (a1) r.a1 += src * step1;
        if (items) r.galois = galois_of(items[i].rot, log_n);
        return r;
    }
    template <int E>
    __device__ void loadv(const LaunchMap& M, int l, int j, PrimeC pc, uint32_t (&x)[E]) const
    {
        const size_t off = (size_t)M.in_off[l] << log_n;
        if constexpr (OWN == Own::Tensor) {
            uint32_t y[E];
            loadv_u32<E>(a0 + off + j, x);
            loadv_u32<E>(a1 + off + j, y);
#pragma unroll
            for (int k = 0; k < E; k++) x[k] = mont(x[k], y[k], pc.q, pc.qinv);
        } else if constexpr (OWN == Own::Plain) {
            loadv_u32<E>(a0 + off + j, x);
        } else {
#pragma unroll
            for (int k = 0; k < E; k++) x[k] = a0[off + aut_src(j + k, galois, log_n)];
        }
    }
    __device__ void load16(const LaunchMap& M, int l, int j, PrimeC pc, uint32_t (&x)[16]) const
    {
        loadv<16>(M, l, j, pc, x);
    }
};

// [t]_q of a lifted (centred) limb stored in the tile-thread layout (rescale)
struct LdCentred {
    static constexpr bool kTileThread = true;
    const int32_t* t;
    int log_n;
    size_t step = 0;
    __device__ LdCentred at(int i) const
    {
        LdCentred r = *this;
        r.t += (size_t)i * step;
        return r;
    }
    __device__ void load16(const LaunchMap& M, int l, int j, PrimeC pc, uint32_t (&x)[16]) const
    {
        load16_u32(reinterpret_cast<const uint32_t*>(t) + ((size_t)M.in_off[l] << log_n) + j, x);
#pragma unroll
        for (int k = 0; k < 16; k++) x[k] = reduce_centred((int32_t)x[k], pc.q);
    }
};

// ---------------------------------------------------------------------------
// storers
// ---------------------------------------------------------------------------
struct StPlain {
    static constexpr bool kTileThread = false;
    uint32_t* base;
    const uint4* fc;  // final constant table (inverse passes), row cidx[l]
    int log_n;
    size_t step = 0;
    __device__ StPlain at(int i) const
    {
        StPlain r = *this;
        r.base += (size_t)i * step;
        return r;
    }
    __device__ void store(const LaunchMap& M, int l, int j, uint32_t v, PrimeC) const
    {
        base[((size_t)M.out_off[l] << log_n) + j] = v;
    }
    __device__ void store16(const LaunchMap& M, int l, int j, const uint32_t (&x)[16], PrimeC) const
    {
        store16_u32(base + ((size_t)M.out_off[l] << log_n) + j, x);
    }
    template <int E>
    __device__ void storev(const LaunchMap& M, int l, int j, const uint32_t (&x)[E], PrimeC) const
    {
        storev_u32<E>(base + ((size_t)M.out_off[l] << log_n) + j, x);
    }
    // epilogue operands requested ahead of the pass: none
    struct Pre {};
    template <int E>
    __device__ Pre prefetch(const LaunchMap&, int, int) const { return {}; }
    template <int E>
    __device__ void storev(const LaunchMap& M, int l, int j, const uint32_t (&x)[E], PrimeC pc, Pre) const
    {
        storev<E>(M, l, j, x, pc);
    }
    __device__ uint4 final_const(const LaunchMap& M, int l) const { return fc[M.cidx[l]]; }
};

// centred lift into int32 (input of a base conversion), tile-thread layout
struct StLift {
    static constexpr bool kTileThread = true;
    int32_t* base;
    const uint4* fc;
    int log_n;
    size_t step = 0;
    __device__ StLift at(int i) const
    {
        StLift r = *this;
        r.base += (size_t)i * step;
        return r;
    }
    template <int E>
    __device__ void storev(const LaunchMap& M, int l, int j, const uint32_t (&x)[E], PrimeC pc) const
    {
        uint32_t y[E];
#pragma unroll
        for (int k = 0; k < E; k++) y[k] = (uint32_t)lift(x[k], pc.q);
        storev_u32<E>(reinterpret_cast<uint32_t*>(base) + ((size_t)M.out_off[l] << log_n) + j, y);
    }
    __device__ void store16(const LaunchMap& M, int l, int j, const uint32_t (&x)[16], PrimeC pc) const
    {
        storev<16>(M, l, j, x, pc);
    }
    __device__ uint4 final_const(const LaunchMap& M, int l) const { return fc[M.cidx[l]]; }
};

// out = (sub - v) * c  (ModDown: c = P^-1 R^2; rescale: c = q_last^-1); sub = 0 where sub_off < 0
struct StCombine {
    static constexpr bool kTileThread = false;
    uint32_t* out0;
    uint32_t* out1;
    const uint32_t* sub;
    const uint2* cst;
    int log_n;
    size_t out_step = 0, sub_step = 0;
    __device__ StCombine at(int i) const
    {
        StCombine r = *this;
        r.out0 += (size_t)i * out_step;
        r.out1 += (size_t)i * out_step;
        r.sub += (size_t)i * sub_step;
        return r;
    }
    // the subtrahend row and the constant, requested ahead of the pass
    template <int E>
    struct PreE {
        uint32_t s[E];
        uint2 c;
    };
    template <int E>
    __device__ PreE<E> prefetch(const LaunchMap& M, int l, int j) const
    {
        PreE<E> p;
        if (M.sub_off[l] >= 0) {
            loadv_u32<E>(sub + ((size_t)M.sub_off[l] << log_n) + j, p.s);
        } else {  // an output prime the input did not have (rational rescaling's added primes)
#pragma unroll
            for (int k = 0; k < E; k++) p.s[k] = 0;
        }
        p.c = cst[M.cidx[l]];
        return p;
    }
    template <int E>
    __device__ void storev(const LaunchMap& M, int l, int j, const uint32_t (&x)[E], PrimeC pc,
                           const PreE<E>& p) const
    {
        uint32_t o[E];
#pragma unroll
        for (int k = 0; k < E; k++) o[k] = mulc(p.s[k] + pc.q - x[k], p.c, pc.q);
        storev_u32<E>((M.grp[l] ? out1 : out0) + ((size_t)M.out_off[l] << log_n) + j, o);
    }
    template <int E>
    __device__ void storev(const LaunchMap& M, int l, int j, const uint32_t (&x)[E], PrimeC pc) const
    {
        storev<E>(M, l, j, x, pc, prefetch<E>(M, l, j));
    }
    __device__ void store16(const LaunchMap& M, int l, int j, const uint32_t (&x)[16], PrimeC pc) const
    {
        storev<16>(M, l, j, x, pc);
    }
};

// ---------------------------------------------------------------------------
// BConv matrix multiplication feeding the NTT column pass (ModUp, ModDown).
// A work-group owns one column tile and up to TPW target primes that share
// their input rows (a digit's lifted rows, or one polynomial's lifted P
// rows).  The input rows stream through registers one at a time into int64
// accumulators of all TPW targets (lazy reduction, Sec. 4.2); each target
// is then reduced once (signed Montgomery), runs the column pass and is
// stored.  Column tile t runs on XCD t mod 8 for every target, so the
// reloads of a tile's inputs by other work-groups hit that XCD's L2.
// ---------------------------------------------------------------------------
// acc - t 2^32 if acc >= t 2^31, acc + t 2^32 if acc < -t 2^31, else acc.
// Adding a multiple of 2^32 touches only the high word, so the fix is a
// select of -t / t / 0 added there (no branch, no 64-bit add).
__device__ __forceinline__ int64_t range_fix(int64_t acc, int64_t t31, int64_t t32)
{
    const int32_t t = (int32_t)(t32 >> 32);
    int32_t adj = acc >= t31 ? -t : 0;
    adj = acc < -t31 ? t : adj;
    const uint32_t hi = (uint32_t)(acc >> 32) + (uint32_t)adj;
    return (int64_t)(((uint64_t)hi << 32) | (uint32_t)acc);
}

// Fused rescale (RS): the group's input rows are followed in y by row e =
// INTT(ks_{l-1}) P^-1 (lifted); the kernel also converts the P rows to
// q_{l-1} (times P^-1), forms t = lift(e - conv_{l-1} P^-1), which is the
// coefficient form of the ModDown output's last limb, and adds t * P to
// every target before the NTT, so the row pass can divide by P q_{l-1}.
struct BcRescale {
    const int32_t* mlast;  // [n_q][n_p] centred [Phat_k P^-1 R]_{q_i}; row l-1 is used
    const int32_t* pr;     // [n_q] centred [P R^-1]_{q_i}, indexed by target prime
    int n_p;
    int level;             // single operation: its level; batched: taken from the item
};

struct BcByPtr {
    const BcMap* p;
    __device__ const BcMap* get() const { return p; }
};
struct BcDir {
    const BcMap* const* dir;
    const BatchItem* items;
    int lo, hi, n_keys, n_src;
    __device__ const BcMap* get() const
    {
        const BatchItem it = items[blockIdx.z];
        return item_ok(it, lo, hi, n_keys, n_src) ? dir[it.level] : nullptr;
    }
};

// A BConv map read through a global-memory pointer: its wave-uniform fields
// then load through the scalar cache into SGPRs.  A map found in a launch
// directory arrives as a generic pointer read from memory, whose fields the
// compiler would otherwise read per lane, into VGPRs, with divergent branches
// on them.
using GlobalBcMap = const __attribute__((address_space(1))) BcMap;

template <int LOG1, int TPW, int NIN, bool RS, class BS, int CT = NTT_THREADS>
__global__ void __launch_bounds__(CT) k_bconv_ntt_cols(NttTables T, BS bs, const int32_t* y0,
                                                                const int32_t* mat, uint32_t* out0, BcRescale X,
                                                                size_t step, const BatchItem* items)
{
    const BcMap* Bp = bs.get();
    if (!Bp) return;
    GlobalBcMap& B = *(GlobalBcMap*)Bp;
    if ((int)blockIdx.y >= B.groups) return;
    const int32_t* y = y0 + (size_t)blockIdx.z * step;
    uint32_t* out = out0 + (size_t)blockIdx.z * step;
    using G = ColGeom<LOG1, CT>;
    __shared__ uint32_t lds[G::LDS];
    const int g = blockIdx.y;
    const int c = threadIdx.x % G::C, r = threadIdx.x / G::C;
    const int tile = col_tile<LOG1, CT>(T.xcd_pair);
    const int col = tile * G::C + c;
    const int n_in = B.n_in[g], n_tg = B.n_tg[g], first = B.first[g];
    const size_t n = (size_t)1 << T.log_n;
    // inputs in the tile-thread layout: this thread's 16 residues of row s
    // are contiguous at s*N + tile*4096 + tid*16
    const int32_t* src = y + (size_t)B.in_off[g] * n + tile * G::TILE + threadIdx.x * 16;

    int64_t acc[TPW][16];
    int64_t t31[TPW], t32[TPW];
#pragma unroll
    for (int t = 0; t < TPW; t++) {
        const int tt = first + (t < n_tg ? t : 0);
        const uint32_t q = T.mods[B.pid[tt]];
        t31[t] = (int64_t)q << 31, t32[t] = (int64_t)q << 32;
#pragma unroll
        for (int k = 0; k < 16; k++) acc[t][k] = 0;
    }
    int64_t accl[RS ? 16 : 1];
    uint32_t ql = 0;
    int64_t l31 = 0, l32 = 0;
    const int ql_pid = RS ? (items ? items[blockIdx.z].level : X.level) - 1 : 0;  // prime id of q_{l-1}
    const int32_t* mlast = X.mlast + (size_t)ql_pid * X.n_p;
    if constexpr (RS) {
        ql = T.mods[ql_pid];
        l31 = (int64_t)ql << 31, l32 = (int64_t)ql << 32;
#pragma unroll
        for (int k = 0; k < 16; k++) accl[k] = 0;
    }
    // one input row at a time (this thread's 16 residues are one 64-byte run);
    // the next row's load is in flight while this row is accumulated
    auto mac = [&](const uint32_t (&yv)[16], int s) {
        if (s >= 8 && (s & 3) == 0) {
#pragma unroll
            for (int t = 0; t < TPW; t++)
#pragma unroll
                for (int k = 0; k < 16; k++) acc[t][k] = range_fix(acc[t][k], t31[t], t32[t]);
            if constexpr (RS) {
#pragma unroll
                for (int k = 0; k < 16; k++) accl[k] = range_fix(accl[k], l31, l32);
            }
        }
#pragma unroll
        for (int t = 0; t < TPW; t++) {
            const int64_t mt = t < n_tg ? mat[B.mat_off[first + t] + s] : 0;
#pragma unroll
            for (int k = 0; k < 16; k++) acc[t][k] += (int64_t)(int32_t)yv[k] * mt;
        }
        if constexpr (RS) {
            const int64_t mt = mlast[s];
#pragma unroll
            for (int k = 0; k < 16; k++) accl[k] += (int64_t)(int32_t)yv[k] * mt;
        }
    };
    uint32_t e[RS ? 16 : 1];
    if constexpr (RS) load16_u32(reinterpret_cast<const uint32_t*>(src + n_in * n), e);  // last limb, used below
    {
        uint32_t ya[16], yb[16];
        if (n_in > 0) load16_u32(reinterpret_cast<const uint32_t*>(src), ya);
        int s = 0;
        for (; s + 1 < n_in; s += 2) {
            load16_u32(reinterpret_cast<const uint32_t*>(src + (s + 1) * n), yb);
            mac(ya, s);
            if (s + 2 < n_in) load16_u32(reinterpret_cast<const uint32_t*>(src + (s + 2) * n), ya);
            mac(yb, s + 1);
        }
        if (s < n_in) mac(ya, s);
    }
    int32_t tl[RS ? 16 : 1];
    if constexpr (RS) {
        const uint32_t qlinv = T.qinvs[ql_pid];
#pragma unroll
        for (int k = 0; k < 16; k++) {
            const uint32_t cl = canon_signed(smr64(range_fix(accl[k], l31, l32), ql, qlinv), ql);
            const int32_t ei = (int32_t)e[k];
            const uint32_t ec = ei < 0 ? (uint32_t)(ei + (int32_t)ql) : (uint32_t)ei;
            tl[k] = lift(sub_mod(ec, cl, ql), ql);
        }
    }

#pragma unroll
    for (int t = 0; t < TPW; t++) {
        if (t >= n_tg) break;
        const int tg = first + t;
        const int pid = B.pid[tg];
        const uint32_t q = T.mods[pid], qinv = T.qinvs[pid];
        const uint2* tw = T.tw + ((size_t)pid << T.log_n);
        uint32_t x[16];
        if constexpr (RS) {
            const int64_t mp = X.pr[pid];
#pragma unroll
            for (int k = 0; k < 16; k++) acc[t][k] = range_fix(acc[t][k], t31[t], t32[t]) + (int64_t)tl[k] * mp;
        }
#pragma unroll
        for (int k = 0; k < 16; k++) x[k] = canon_signed(smr64(range_fix(acc[t][k], t31[t], t32[t]), q, qinv), q);
        uint32_t* dst = out + (size_t)B.out_off[tg] * n + col;
        by_class(q, [&](auto tag) {
            constexpr bool W = decltype(tag)::value;
            ct_stages<4, W>(x, q, [&](int u, int b) { return tw[(1 << u) + b]; });
            if constexpr (G::NS2 > 0) {
                if (t) __syncthreads();  // previous target's LDS reads are done
#pragma unroll
                for (int k = 0; k < 16; k++) lds[col_lds<G::C>(r + G::R * k, c)] = x[k];
                __syncthreads();
#pragma unroll
                for (int k = 0; k < 16; k++) x[k] = lds[col_lds<G::C>(16 * r + k, c)];
                ct_stages<G::NS2, W>(x, q, [&](int u, int b) {
                    return tw[(1 << (4 + u)) + (r << (4 - G::NS2 + u)) + b];
                });
            }
        });
        if constexpr (G::NS2 > 0) {
#pragma unroll
            for (int k = 0; k < 16; k++) dst[(16 * r + k) * ROW] = x[k];
        } else {
#pragma unroll
            for (int k = 0; k < 16; k++) dst[(r + G::R * k) * ROW] = x[k];
        }
    }
}

// ---------------------------------------------------------------------------
// BConv + NTT column pass with 4 residues per thread (Col4 geometry; lifted
// inputs in the 4-residue tile-thread layout of k_inv_cols4).  The group's
// input rows are requested together (four at a time: 54-56 VGPRs, 8
// work-groups per CU; eight at a time needs 74-80), with its matrix
// constants and its targets' twiddles (staged in LDS); the TPW targets'
// column transforms then run round by round together, one barrier per
// exchange.  Same residues as k_bconv_ntt_cols.
// ---------------------------------------------------------------------------
template <int LOG1, int TPW, bool RS, class BS>
__global__ void __launch_bounds__(NTT_THREADS) k_bconv_ntt_cols4(NttTables T, BS bs, const int32_t* y0,
                                                                  const int32_t* mat, uint32_t* out0, BcRescale X,
                                                                  size_t step, const BatchItem* items)
{
    using G = Col4<LOG1>;
    constexpr int CH = 4;  // input rows in flight (<= BCONV_MAT_PAD)
    const BcMap* Bp = bs.get();
    if (!Bp) return;
    GlobalBcMap& B = *(GlobalBcMap*)Bp;
    const int g = blockIdx.y;  // grid.y <= MAX_BC_GROUPS: the entries read below are in bounds
    const int groups = B.groups, n_in = B.n_in[g], n_tg = B.n_tg[g], first = B.first[g], in_off = B.in_off[g];
    if (g >= groups) return;
    const int32_t* y = y0 + (size_t)blockIdx.z * step;
    uint32_t* out = out0 + (size_t)blockIdx.z * step;
    __shared__ uint32_t lds[TPW * G::WORDS];
    __shared__ uint2 twl[TPW << LOG1];
    const int c = threadIdx.x % G::C, t = threadIdx.x / G::C;
    const int tile = col4_tile<LOG1>(T.xcd_pair), col = tile * G::C + c;
    const size_t n = (size_t)1 << T.log_n;
    // the group's input rows start at ybase (uniform); this thread's four
    // residues sit at toff in each (a 32-bit offset from a scalar base)
    const uint32_t* ybase = reinterpret_cast<const uint32_t*>(y + (size_t)in_off * n + tile * G::TILE);
    const uint32_t toff = threadIdx.x * 4;

    // targets (a group's missing targets repeat its first; they are not stored)
    uint32_t tq[TPW], tqi[TPW];
    const uint2* tws[TPW];
    const int32_t* tm[TPW];
    int64_t t31[TPW], t32[TPW];
#pragma unroll
    for (int i = 0; i < TPW; i++) {
        const int k = first + (i < n_tg ? i : 0);
        const int pid = B.pid[k];
        tq[i] = T.mods[pid], tqi[i] = T.qinvs[pid];
        tws[i] = T.tw + ((size_t)pid << T.log_n);
        tm[i] = mat + B.mat_off[k];
        t31[i] = (int64_t)tq[i] << 31, t32[i] = (int64_t)tq[i] << 32;
    }
    // fused rescale: row e (after the inputs) and the conversion to q_{l-1}
    const int ql_pid = RS ? (items ? items[blockIdx.z].level : X.level) - 1 : 0;
    const int32_t* mlast = X.mlast + (size_t)ql_pid * X.n_p;
    uint32_t e[RS ? 4 : 1];
    if constexpr (RS) loadv_u32<4>(ybase + (size_t)n_in * n + toff, e);
    uint32_t yv[CH][4];
    auto load_rows = [&](int s0) {  // rows past the inputs repeat the last one (their constants are zero)
#pragma unroll
        for (int s = 0; s < CH; s++) loadv_u32<4>(ybase + (size_t)min(s0 + s, n_in - 1) * n + toff, yv[s]);
    };
    if (n_in > 0) load_rows(0);
    col4_stage_twiddles<LOG1, TPW>(twl, tws);

    int64_t acc[TPW][4];
#pragma unroll
    for (int i = 0; i < TPW; i++)
#pragma unroll
        for (int k = 0; k < 4; k++) acc[i][k] = 0;
    int64_t accl[RS ? 4 : 1];
    uint32_t ql = 0;
    int64_t l31 = 0, l32 = 0;
    if constexpr (RS) {
        ql = T.mods[ql_pid];
        l31 = (int64_t)ql << 31, l32 = (int64_t)ql << 32;
#pragma unroll
        for (int k = 0; k < 4; k++) accl[k] = 0;
    }
    // Chunks of CH input rows: the chunk's matrix constants are requested
    // together, zero past the group's inputs (every matrix ends with CH spare
    // entries, so those reads stay in bounds), so a chunk is CH multiply-adds
    // per residue without branches.  A group's missing targets accumulate its
    // first target's row, unstored.  The first chunk (the only one when a
    // digit has at most CH primes) runs straight from the rows loaded above.
    auto mac_chunk = [&](int s0) {
        int32_t mv[TPW][CH], ml[RS ? CH : 1];
#pragma unroll
        for (int s = 0; s < CH; s++) {
            const bool in = s0 + s < n_in;
#pragma unroll
            for (int i = 0; i < TPW; i++) {
                const int32_t m = tm[i][s0 + s];
                mv[i][s] = in ? m : 0;
            }
            if constexpr (RS) {
                const int32_t m = mlast[s0 + s];
                ml[s] = in ? m : 0;
            }
        }
#pragma unroll
        for (int s1 = 0; s1 < CH; s1++) {
            if ((s1 & 3) == 0 && s0 + s1 >= 8) {  // lazy reduction: range fix after 8 products, then every 4
#pragma unroll
                for (int i = 0; i < TPW; i++)
#pragma unroll
                    for (int k = 0; k < 4; k++) acc[i][k] = range_fix(acc[i][k], t31[i], t32[i]);
                if constexpr (RS) {
#pragma unroll
                    for (int k = 0; k < 4; k++) accl[k] = range_fix(accl[k], l31, l32);
                }
            }
#pragma unroll
            for (int i = 0; i < TPW; i++)
#pragma unroll
                for (int k = 0; k < 4; k++) acc[i][k] += (int64_t)(int32_t)yv[s1][k] * (int64_t)mv[i][s1];
            if constexpr (RS) {
#pragma unroll
                for (int k = 0; k < 4; k++) accl[k] += (int64_t)(int32_t)yv[s1][k] * (int64_t)ml[s1];
            }
        }
    };
    if (n_in > 0) mac_chunk(0);
    for (int s0 = CH; s0 < n_in; s0 += CH) {
        load_rows(s0);
        mac_chunk(s0);
    }
    int32_t tl[RS ? 4 : 1];
    if constexpr (RS) {
        const uint32_t qlinv = T.qinvs[ql_pid];
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const uint32_t cl = canon_signed(smr64(range_fix(accl[k], l31, l32), ql, qlinv), ql);
            const int32_t ei = (int32_t)e[k];
            const uint32_t ec = ei < 0 ? (uint32_t)(ei + (int32_t)ql) : (uint32_t)ei;
            tl[k] = lift(sub_mod(ec, cl, ql), ql);
        }
    }
    uint32_t x[TPW][4];
#pragma unroll
    for (int i = 0; i < TPW; i++) {
        int64_t mp = 0;
        if constexpr (RS) mp = X.pr[B.pid[first + (i < n_tg ? i : 0)]];
#pragma unroll
        for (int k = 0; k < 4; k++) {
            int64_t a = acc[i][k];
            if constexpr (RS) a = range_fix(a, t31[i], t32[i]) + (int64_t)tl[k] * mp;
            x[i][k] = canon_signed(smr64(range_fix(a, t31[i], t32[i]), tq[i], tqi[i]), tq[i]);
        }
    }
    col4_fwd<LOG1, TPW>(x, tq, lds, twl, c, t);
#pragma unroll
    for (int i = 0; i < TPW; i++) {
        if (i >= n_tg) break;
        uint32_t* dst = out + (size_t)B.out_off[first + i] * n + col;
#pragma unroll
        for (int k = 0; k < 4; k++) dst[(size_t)(4 * t + k) * ROW] = x[i][k];
    }
}

// ---------------------------------------------------------------------------
// KeyMult (Sec. 2.3; Par.1): one output row r of R_{Q_l P} for all digits.
// For each digit j: the digit's own rows come straight from the input; every
// other row finishes its ModUp NTT here (row pass) and is multiplied into the
// accumulators with evk_j.  Q rows then take the HMult / HRot term times P
// and are stored; P rows run ModDown's INTT row pass and are stored.
// All accumulated values carry a factor 2^-64 (two Montgomery products),
// removed by ModDown's constants.
// ---------------------------------------------------------------------------
struct KmArgs {
    const uint32_t* up;   // ModUp column-pass output: digit j, row r at (j*(level+alpha) + r) * N
    const uint32_t* evk;  // [dnum][2][n_q+n_p][N]
    const uint32_t* b0;
    const uint32_t* a0;
    const uint32_t* b1;
    const uint32_t* a1;
    uint32_t* ks_q;       // [2][level][N]
    uint32_t* ks_p;       // [2][n_p + rs][N] (after the INTT row pass)
    const uint32_t* p_mod_q;
    const uint2* rinv;
    const uint2* p_r2;
    const uint2* r1;      // [n_q + n_p] x -> x 2^32 (folds a 64-bit KeyMult sum, k_keymult4)
    uint32_t galois;
    int level, n_q, n_p;
    int base;             // prime id of the level's first limb (a window of the list; 0 in batched launches)
    int rs;               // rows dropped by a rescaling that follows (0: none): they take the INTT row
                          // pass into slots n_p.. of ks_p, in row order
    int dlo, dhi;         // rows kept by that rescaling: [dlo, dhi) (dhi < 0: level - 1, single rescaling)
    const int32_t* lv;    // batched launch on a windowed context: per-level window data (Ctx::lv_tab)
    // batched launch (items != nullptr): item blockIdx.z takes its level, key
    // and Galois element from items and advances the pointers by these steps;
    // an item whose level is outside [lo_level, level] or whose key index is
    // outside [0, n_keys) is skipped
    const BatchItem* items;
    size_t in_step, in2_step, ws_step, key_step, up_step;
    int lo_level, n_keys, n_src;
};

// End of a KeyMult row: Q rows store ks; P rows (and the dropped row q_{l-1}
// when rescale follows) start ModDown with the INTT row pass, then store.
template <int LOG1>
__device__ __forceinline__ void keymult_store(const NttTables& Ti, const KmArgs& A, int r, int pid, int h, int rp,
                                              int rr, uint32_t q, uint32_t* lds, const uint32_t (&acc0)[16],
                                              const uint32_t (&acc1)[16])
{
    const int log_n = Ti.log_n;
    const size_t n = (size_t)1 << log_n;
    const int j0 = h * ROW + 16 * rp;
    const int dhi = A.dhi < 0 ? A.level - 1 : A.dhi;
    const bool dropped = A.rs && r < A.level && (r < A.dlo || r >= dhi);
    const bool to_coef = r >= A.level || dropped;
    if (!to_coef) {
        store16_u32(A.ks_q + (size_t)r * n + j0, acc0);
        store16_u32(A.ks_q + ((size_t)A.level + r) * n + j0, acc1);
    } else {
        const uint2* twi = Ti.tw + ((size_t)pid << log_n);
        const int slot = r >= A.level ? r - A.level : A.n_p + (r < A.dlo ? r : A.dlo + (r - dhi));
#pragma unroll
        for (int poly = 0; poly < 2; poly++) {
            uint32_t x[16];
#pragma unroll
            for (int k = 0; k < 16; k++) x[k] = poly ? acc1[k] : acc0[k];
            by_class(q, [&](auto tag) {
                constexpr bool W = decltype(tag)::value;
                gs_stages<4, W, false>(x, q, [&](int u, int b) {
                    return twi[(1 << (LOG1 + 4 + u)) + (h << (4 + u)) + (rp << u) + b];
                });
#pragma unroll
                for (int k = 0; k < 16; k++) lds[row_lds(rr, 16 * rp + k)] = x[k];
                __syncthreads();
#pragma unroll
                for (int k = 0; k < 16; k++) x[k] = lds[row_lds(rr, rp + 16 * k)];
                __syncthreads();
                gs_stages<4, W, false>(x, q, [&](int u, int b) { return twi[(1 << (LOG1 + u)) + (h << u) + b]; });
            });
            uint32_t* dst = A.ks_p + ((size_t)poly * (A.n_p + A.rs) + slot) * n + (size_t)h * ROW;
#pragma unroll
            for (int k = 0; k < 16; k++) dst[rp + 16 * k] = x[k];
        }
    }
}

// Batched KeyMult launch: item blockIdx.z's level, window, key, rotation and
// pointers replace the launch's; false if the item is skipped.
__device__ __forceinline__ bool km_item(KmArgs& A, int log_n)
{
    if (!A.items) return true;
    const BatchItem it = A.items[blockIdx.z];
    const size_t z = blockIdx.z;
    if (!item_ok(it, A.lo_level, A.level, A.n_keys, A.n_src)) return false;
    A.level = it.level;
    if (A.lv) {  // windowed context: the item's window, and its rescaling's dropped rows
        constexpr int S = MAX_PRIMES + 1;
        A.base = A.lv[it.level];
        if (A.base < 0) return false;  // no window with this many limbs
        if (A.rs) {
            A.rs = A.lv[S + it.level];
            if (A.rs == 0) return false;  // no window below to rescale to
            A.dlo = A.lv[2 * S + it.level];
            A.dhi = A.lv[3 * S + it.level];
        }
    }
    A.galois = galois_of(it.rot, log_n);
    A.evk += (size_t)it.key * A.key_step;
    const size_t src = (size_t)it.src;  // input slot
    A.b0 += src * A.in_step;
    A.a0 += src * A.in_step;
    if (A.b1) A.b1 += src * A.in2_step;
    if (A.a1) A.a1 += src * A.in2_step;
    A.up += z * A.up_step;
    A.ks_q += z * A.ws_step;
    A.ks_p += z * A.ws_step;
    return true;
}

template <int LOG1, Own OWN, Extra EX>
__global__ void __launch_bounds__(NTT_THREADS) k_keymult(NttTables Tf, NttTables Ti, KmArgs A)
{
    __shared__ uint32_t lds[ROW_LDS_WORDS];
    if (!km_item(A, Tf.log_n)) return;
    const int r = blockIdx.y;  // row in q_b..q_{b+l-1}, p_0..
    if (r >= A.level + A.n_p) return;
    // window digit j is the part of key digit kd + j inside the window;
    // the window starts woff primes into key digit kd
    const int woff = A.base % A.n_p, kd = A.base / A.n_p;
    const int beta = (woff + A.level + A.n_p - 1) / A.n_p;
    const int log_n = Tf.log_n;
    const int pid = r < A.level ? A.base + r : A.n_q + (r - A.level);  // also the key row
    const uint32_t q = Tf.mods[pid], qinv = Tf.qinvs[pid];
    const int rp = threadIdx.x % 16, rr = threadIdx.x / 16;
    const int h = blockIdx.x * ROWS_PER_WG + rr;
    const int j0 = h * ROW + 16 * rp;
    const size_t n = (size_t)1 << log_n;
    const uint2* twf = Tf.tw + ((size_t)pid << log_n);
    const int rows = A.level + A.n_p, key_rows = A.n_q + A.n_p;

    uint32_t acc0[16], acc1[16];
#pragma unroll
    for (int k = 0; k < 16; k++) acc0[k] = acc1[k] = 0;

    // The row's prime is the same for every digit: its row-pass twiddles are
    // generated into LDS once, ahead of the digit loop.
    __shared__ uint2 tws[OWN == Own::Hoisted ? 1 : ROWS_PER_WG * ROW_TW_SLOTS];
    if constexpr (OWN != Own::Hoisted) stage_row_twiddles<LOG1>(tws, twf, blockIdx.x * ROWS_PER_WG, q);

    for (int j = 0; j < beta; j++) {
        // this digit's key rows are loaded first and arrive while x is formed
        uint32_t kb[16], ka[16];
        load16_u32(A.evk + ((size_t)(2 * (kd + j)) * key_rows + pid) * n + j0, kb);
        load16_u32(A.evk + ((size_t)(2 * (kd + j) + 1) * key_rows + pid) * n + j0, ka);
        uint32_t x[16];
        const int lo = max(j * A.n_p - woff, 0), hi = min((j + 1) * A.n_p - woff, A.level);
        if (r >= lo && r < hi) {
            const size_t off = (size_t)r * n;
            if constexpr (OWN == Own::Tensor) {
                uint32_t y[16];
                load16_u32(A.a0 + off + j0, x);
                load16_u32(A.a1 + off + j0, y);
                if constexpr (EX == Extra::HMult) {
                    // + P*d0, + P*d1 (d0 = b_a b_b, d1 = b_a a_b + a_a b_b) while a_a, a_b
                    // are in registers: this row's inputs are read once
                    uint32_t ba[16], bb[16];
                    load16_u32(A.b0 + off + j0, ba);
                    load16_u32(A.b1 + off + j0, bb);
                    const uint32_t pq = A.p_mod_q[pid];
#pragma unroll
                    for (int k = 0; k < 16; k++) {
                        const uint32_t d0 = mont(ba[k], bb[k], q, qinv);
                        const uint32_t d1 = add_mod(mont(ba[k], y[k], q, qinv), mont(x[k], bb[k], q, qinv), q);
                        acc0[k] = add_mod(acc0[k], mont(d0, pq, q, qinv), q);
                        acc1[k] = add_mod(acc1[k], mont(d1, pq, q, qinv), q);
                    }
                }
#pragma unroll
                for (int k = 0; k < 16; k++) x[k] = mont(x[k], y[k], q, qinv);
            } else {
                if constexpr (OWN == Own::Plain) {
                    load16_u32(A.a0 + off + j0, x);
                } else {  // Gather, Hoisted: phi_g(a)
#pragma unroll
                    for (int k = 0; k < 16; k++) x[k] = A.a0[off + aut_src(j0 + k, A.galois, log_n)];
                }
                const uint2 c = A.rinv[pid];
#pragma unroll
                for (int k = 0; k < 16; k++) x[k] = mulc(x[k], c, q);
            }
        } else if constexpr (OWN == Own::Hoisted) {
            // ModUp row already in the evaluation domain: gather phi_g on load
            const uint32_t* src = A.up + (size_t)(j * rows + r) * n;
#pragma unroll
            for (int k = 0; k < 16; k++) x[k] = src[aut_src(j0 + k, A.galois, log_n)];
        } else {
            const uint32_t* src = A.up + (size_t)(j * rows + r) * n + (size_t)h * ROW;
#pragma unroll
            for (int k = 0; k < 16; k++) x[k] = src[rp + 16 * k];
            by_class(q, [&](auto tag) {
                constexpr bool W = decltype(tag)::value;
                ct_stages<4, W>(x, q, [&](int u, int b) { return row_tw1(tws, rr, u, b); });
#pragma unroll
                for (int k = 0; k < 16; k++) lds[row_lds(rr, rp + 16 * k)] = x[k];
                __syncthreads();
#pragma unroll
                for (int k = 0; k < 16; k++) x[k] = lds[row_lds(rr, 16 * rp + k)];
                __syncthreads();
                ct_stages<4, W>(x, q, [&](int u, int b) { return row_tw2(tws, rr, rp, u, b); });
            });
        }
#pragma unroll
        for (int k = 0; k < 16; k++) {
            acc0[k] = add_mod(acc0[k], mont(x[k], kb[k], q, qinv), q);
            acc1[k] = add_mod(acc1[k], mont(x[k], ka[k], q, qinv), q);
        }
    }

    if (r < A.level) {
        if constexpr (EX == Extra::HRot) {
            const uint2 c = A.p_r2[pid];
#pragma unroll
            for (int k = 0; k < 16; k++)
                acc0[k] = add_mod(acc0[k], mulc(A.b0[(size_t)r * n + aut_src(j0 + k, A.galois, log_n)], c, q), q);
        }
    }
    keymult_store<LOG1>(Ti, A, r, pid, h, rp, rr, q, lds, acc0, acc1);
}

// ---------------------------------------------------------------------------
// KeyMult with one wave per 256-point row (4 residues per thread, ROWS4 rows
// per work-group): four times the waves of k_keymult, for launches with few
// rows in flight.  Same inputs, outputs and residues as k_keymult.
//  * The ModUp rows finish their NTT row pass as four radix-4 rounds with
//    three exchanges through the wave's own LDS rows (as k_fwd_rows4); the
//    row's twelve twiddles per thread stay in registers across the digits.
//  * The digit products of a coefficient (each below q^2 < 2^62) are summed
//    exactly in 64 bits and reduced once: x 2^-32 of the sum is the same
//    residue as the sum of per-digit Montgomery products.  At most four
//    products (or a folded value and three products) are summed before a
//    fold (hi 2^32 + lo -> [hi 2^32]_q + lo), which keeps the sum below
//    2q 2^32, the input range of redc64.
//  * P rows (and the rows a following rescaling drops) run ModDown's INTT
//    row pass the same way before they are stored.
// ---------------------------------------------------------------------------
// sum x 2^-32 mod q for a sum below 2q 2^32 (odd q < 2^31, qinv = q^-1 mod
// 2^32): m = lo qinv makes sum - m q divisible by 2^32 with equal low words,
// so the quotient is hi - mulhi(m, q), in (-q, 2q); two corrections end in
// [0, q).
__device__ __forceinline__ uint32_t redc64(uint64_t sum, uint32_t q, uint32_t qinv)
{
    const uint32_t lo = (uint32_t)sum, hi = (uint32_t)(sum >> 32);
    const uint32_t t = __umulhi(lo * qinv, q);
    const uint32_t r = hi >= t ? hi - t : hi - t + q;
    return red2(r, q);
}

// hi 2^32 + lo -> lo + [hi 2^32]_q (same residue, below 2^32 + q)
__device__ __forceinline__ uint64_t fold64(uint64_t sum, uint2 r1, uint32_t q)
{
    return (uint64_t)(uint32_t)sum + mulc((uint32_t)(sum >> 32), r1, q);
}

template <int LOG1, Own OWN, Extra EX>
__global__ void __launch_bounds__(NTT_THREADS) k_keymult4(NttTables Tf, NttTables Ti, KmArgs A)
{
    __shared__ uint32_t lds[ROWS4 * ROW4_PITCH];
    if (!km_item(A, Tf.log_n)) return;
    // row in q_b..q_{b+l-1}, p_0..: the P rows (the longest work: every digit
    // needs its row pass, then two INTT row passes) take the first grid rows,
    // so they are dispatched first and do not form the launch's tail
    if ((int)blockIdx.y >= A.level + A.n_p) return;
    const int r = ((int)blockIdx.y + A.level) % (A.level + A.n_p);
    const int woff = A.base % A.n_p, kd = A.base / A.n_p;  // as in k_keymult
    const int beta = (woff + A.level + A.n_p - 1) / A.n_p;
    const int log_n = Tf.log_n;
    const int pid = r < A.level ? A.base + r : A.n_q + (r - A.level);  // also the key row
    const uint32_t q = Tf.mods[pid], qinv = Tf.qinvs[pid];
    const int t = threadIdx.x & 63, w = wave_id();
    const int h = blockIdx.x * ROWS4 + w;
    const int j0 = h * ROW + 4 * t;  // this thread's residues: row h, positions 4t .. 4t+3
    // contiguous accesses as a wave-uniform pointer (through row h) plus the
    // lane's 32-bit offset 4t (scalar-base loads and stores)
    const size_t hrow = (size_t)h * ROW;
    const uint32_t l4 = 4u * (uint32_t)t;
    const size_t n = (size_t)1 << log_n;
    const int rows = A.level + A.n_p, key_rows = A.n_q + A.n_p;

    uint2 twf[4][3];
    if constexpr (OWN != Own::Hoisted) row4_twiddles_q<LOG1, false>(Tf.twq + ((size_t)pid << log_n), q, h, t, twf);
    uint64_t s0[4], s1[4];
#pragma unroll
    for (int k = 0; k < 4; k++) s0[k] = s1[k] = 0;
    int terms = 0;  // products in s0 / s1 since the last fold
    const uint2 r1 = A.r1[pid];
    constexpr bool EXTRA = OWN == Own::Tensor && EX == Extra::HMult;

    // The digit whose own rows this row is (none for P rows); its input rows
    // are requested at the start, every digit's key rows and ModUp row one
    // digit ahead of their use.
    int jown = -1;
    for (int j = 0; j < beta; j++)
        if (r >= max(j * A.n_p - woff, 0) && r < min((j + 1) * A.n_p - woff, A.level)) jown = j;
    uint32_t o0[4], o1[4], o2[4], o3[4];  // Tensor: a_a, a_b (and b_a, b_b for HMult); else the input row
    if (jown >= 0) {
        const size_t off = (size_t)r * n;
        if constexpr (OWN == Own::Tensor) {
            loadv_u32<4>(A.a0 + (off + hrow) + l4, o0);
            loadv_u32<4>(A.a1 + (off + hrow) + l4, o1);
            if constexpr (EXTRA) {
                loadv_u32<4>(A.b0 + (off + hrow) + l4, o2);
                loadv_u32<4>(A.b1 + (off + hrow) + l4, o3);
            }
        } else if constexpr (OWN == Own::Plain) {
            loadv_u32<4>(A.a0 + (off + hrow) + l4, o0);
        } else {  // Gather, Hoisted: phi_g(a)
#pragma unroll
            for (int k = 0; k < 4; k++) o0[k] = A.a0[off + aut_src(j0 + k, A.galois, log_n)];
        }
    }
    struct Dig {
        uint32_t kb[4], ka[4], x[4];
    };
    auto issue = [&](int j, Dig& d) {
        loadv_u32<4>(A.evk + (((size_t)(2 * (kd + j)) * key_rows + pid) * n + hrow) + l4, d.kb);
        loadv_u32<4>(A.evk + (((size_t)(2 * (kd + j) + 1) * key_rows + pid) * n + hrow) + l4, d.ka);
        if (j == jown) return;
        if constexpr (OWN == Own::Hoisted) {  // ModUp row already in the evaluation domain: gather phi_g
            const uint32_t* src = A.up + (size_t)(j * rows + r) * n;
#pragma unroll
            for (int k = 0; k < 4; k++) d.x[k] = src[aut_src(j0 + k, A.galois, log_n)];
        } else {
            const uint32_t* src = A.up + (size_t)(j * rows + r) * n + (size_t)h * ROW;
#pragma unroll
            for (int k = 0; k < 4; k++) d.x[k] = src[t + 64 * k];
        }
    };
    // digit j from cur; requests digit j + 1 into nxt first
    auto step = [&](int j, Dig& cur, Dig& nxt) {
        if (j + 1 < beta) issue(j + 1, nxt);
        const bool own = j == jown;
        if (terms + 1 + (EXTRA && own ? 1 : 0) > 4) {  // uniform across the launch
#pragma unroll
            for (int k = 0; k < 4; k++) s0[k] = fold64(s0[k], r1, q), s1[k] = fold64(s1[k], r1, q);
            terms = 1;  // the folded value (below 2^32 + q) counts as one product
        }
        uint32_t x[4];
        if (own) {
            if constexpr (OWN == Own::Tensor) {
                if constexpr (EXTRA) {
                    // P d0 and P d1 (d0 = b_a b_b, d1 = b_a a_b + a_a b_b) join the sums
                    const uint32_t pq = A.p_mod_q[pid];
#pragma unroll
                    for (int k = 0; k < 4; k++) {
                        const uint32_t d0 = mont(o2[k], o3[k], q, qinv);
                        const uint32_t d1 = add_mod(mont(o2[k], o1[k], q, qinv), mont(o0[k], o3[k], q, qinv), q);
                        s0[k] += (uint64_t)d0 * pq;
                        s1[k] += (uint64_t)d1 * pq;
                    }
                    terms++;
                }
#pragma unroll
                for (int k = 0; k < 4; k++) x[k] = mont(o0[k], o1[k], q, qinv);
            } else {
                const uint2 c = A.rinv[pid];
#pragma unroll
                for (int k = 0; k < 4; k++) x[k] = mulc(o0[k], c, q);
            }
        } else {
#pragma unroll
            for (int k = 0; k < 4; k++) x[k] = cur.x[k];
            if constexpr (OWN != Own::Hoisted)
                by_class(q, [&](auto tag) { row4_fwd<decltype(tag)::value>(x, q, lds, w, t, twf); });
        }
#pragma unroll
        for (int k = 0; k < 4; k++) {
            s0[k] += (uint64_t)x[k] * cur.kb[k];
            s1[k] += (uint64_t)x[k] * cur.ka[k];
        }
        terms++;
    };
    Dig da, db;
    issue(0, da);
    for (int j = 0; j < beta; j += 2) {  // two digits per trip: the buffers swap roles without copies
        step(j, da, db);
        if (j + 1 < beta) step(j + 1, db, da);
    }

    uint32_t acc0[4], acc1[4];
#pragma unroll
    for (int k = 0; k < 4; k++) acc0[k] = redc64(s0[k], q, qinv), acc1[k] = redc64(s1[k], q, qinv);
    if (r < A.level) {
        if constexpr (EX == Extra::HRot) {
            const uint2 c = A.p_r2[pid];
#pragma unroll
            for (int k = 0; k < 4; k++)
                acc0[k] = add_mod(acc0[k], mulc(A.b0[(size_t)r * n + aut_src(j0 + k, A.galois, log_n)], c, q), q);
        }
    }

    // Q rows store ks; P rows (and the rows a following rescaling drops) start
    // ModDown with the INTT row pass, then store
    const int dhi = A.dhi < 0 ? A.level - 1 : A.dhi;
    const bool dropped = A.rs && r < A.level && (r < A.dlo || r >= dhi);
    if (r < A.level && !dropped) {
        storev_u32<4>(A.ks_q + ((size_t)r * n + hrow) + l4, acc0);
        storev_u32<4>(A.ks_q + (((size_t)A.level + r) * n + hrow) + l4, acc1);
        return;
    }
    uint2 twi[4][3];
    row4_twiddles_q<LOG1, true>(Ti.twq + ((size_t)pid << log_n), q, h, t, twi);
    const int slot = r >= A.level ? r - A.level : A.n_p + (r < A.dlo ? r : A.dlo + (r - dhi));
#pragma unroll
    for (int poly = 0; poly < 2; poly++) {
        uint32_t x[4];
#pragma unroll
        for (int k = 0; k < 4; k++) x[k] = poly ? acc1[k] : acc0[k];
        by_class(q, [&](auto tag) { row4_inv<decltype(tag)::value>(x, q, lds, w, t, twi); });
        uint32_t* dst = A.ks_p + ((size_t)poly * (A.n_p + A.rs) + slot) * n + (size_t)h * ROW;
#pragma unroll
        for (int k = 0; k < 4; k++) dst[t + 64 * k] = x[k];
    }
}

// ---------------------------------------------------------------------------
// Sum of plaintext-weighted rotations (Sec. 5 Par.4/Par.5, Eq. 5): one
// KeyMult pass over all rotations.  For row r, rotation i: the shared ModUp
// rows (evaluation domain) and the own digit's input row are gathered
// through phi_i, multiplied into rotation i's key rows, weighted by the
// plaintext row pt_i (taken to Montgomery form, so the 2^-64 bookkeeping of
// ks is unchanged) and accumulated; Q rows also take P * pt_i * phi_i(b).
// One ModDown follows.  items[i] = {level, key, rot, -}.
// ---------------------------------------------------------------------------
template <int LOG1>
__global__ void __launch_bounds__(NTT_THREADS) k_keymult_sum(NttTables Tf, NttTables Ti, KmArgs A,
                                                              const uint32_t* pts, size_t pt_step, int n_rot,
                                                              const uint2* rmont)
{
    __shared__ uint32_t lds[ROW_LDS_WORDS];
    const int r = blockIdx.y;
    if (r >= A.level + A.n_p) return;
    const int woff = A.base % A.n_p, kd = A.base / A.n_p;  // as in k_keymult
    const int beta = (woff + A.level + A.n_p - 1) / A.n_p;
    const int log_n = Tf.log_n;
    const int pid = r < A.level ? A.base + r : A.n_q + (r - A.level);  // also the key and plaintext row
    const uint32_t q = Tf.mods[pid], qinv = Tf.qinvs[pid];
    const int rp = threadIdx.x % 16, rr = threadIdx.x / 16;
    const int h = blockIdx.x * ROWS_PER_WG + rr;
    const int j0 = h * ROW + 16 * rp;
    const size_t n = (size_t)1 << log_n;
    const int rows = A.level + A.n_p, key_rows = A.n_q + A.n_p;
    const uint2 cm = rmont[pid];  // x -> x 2^32 mod q

    uint32_t acc0[16], acc1[16];
#pragma unroll
    for (int k = 0; k < 16; k++) acc0[k] = acc1[k] = 0;
    for (int i = 0; i < n_rot; i++) {
        const BatchItem it = A.items[i];
        if (!item_ok(it, A.level, A.level, A.n_keys, 0)) continue;  // uniform across the launch
        const uint32_t g = galois_of(it.rot, log_n);
        const uint32_t* evk = A.evk + (size_t)it.key * A.key_step;
        uint32_t s0[16], s1[16];
#pragma unroll
        for (int k = 0; k < 16; k++) s0[k] = s1[k] = 0;
        for (int j = 0; j < beta; j++) {
            uint32_t kb[16], ka[16], x[16];
            load16_u32(evk + ((size_t)(2 * (kd + j)) * key_rows + pid) * n + j0, kb);
            load16_u32(evk + ((size_t)(2 * (kd + j) + 1) * key_rows + pid) * n + j0, ka);
            const int lo = max(j * A.n_p - woff, 0), hi = min((j + 1) * A.n_p - woff, A.level);
            if (r >= lo && r < hi) {  // the digit's own row: phi(a) times R^-1, as in ModUp's own rows
                const size_t off = (size_t)r * n;
                const uint2 c = A.rinv[pid];
#pragma unroll
                for (int k = 0; k < 16; k++) x[k] = mulc(A.a0[off + aut_src(j0 + k, g, log_n)], c, q);
            } else {
                const uint32_t* src = A.up + (size_t)(j * rows + r) * n;
#pragma unroll
                for (int k = 0; k < 16; k++) x[k] = src[aut_src(j0 + k, g, log_n)];
            }
#pragma unroll
            for (int k = 0; k < 16; k++) {
                s0[k] = add_mod(s0[k], mont(x[k], kb[k], q, qinv), q);
                s1[k] = add_mod(s1[k], mont(x[k], ka[k], q, qinv), q);
            }
        }
        uint32_t pm[16];
        load16_u32(pts + (size_t)i * pt_step + (size_t)pid * n + j0, pm);
#pragma unroll
        for (int k = 0; k < 16; k++) {
            pm[k] = mulc(pm[k], cm, q);  // p 2^32: mont(s, p 2^32) = s p
            acc0[k] = add_mod(acc0[k], mont(s0[k], pm[k], q, qinv), q);
            acc1[k] = add_mod(acc1[k], mont(s1[k], pm[k], q, qinv), q);
        }
        if (r < A.level) {  // + P * p * phi(b), with the R^-2 of ks
            const uint2 c = A.p_r2[pid];
#pragma unroll
            for (int k = 0; k < 16; k++) {
                const uint32_t pb = mulc(A.b0[(size_t)r * n + aut_src(j0 + k, g, log_n)], c, q);
                acc0[k] = add_mod(acc0[k], mont(pb, pm[k], q, qinv), q);
            }
        }
    }
    keymult_store<LOG1>(Ti, A, r, pid, h, rp, rr, q, lds, acc0, acc1);
}

// ---------------------------------------------------------------------------
// stand-alone base conversion (coefficient domain)
// ---------------------------------------------------------------------------
// BConv matrix multiplication with lazy reduction (Sec. 4.2): centred inputs
// y_s (|y_s| < 2^30) times centred constants M_s (|M_s| < t/2) accumulate in
// int64; after 8 products and then after every 4 more, add or subtract
// 2^32 t to stay in [-2^31 t, 2^31 t); one signed Montgomery reduction at the
// end.  The reduction's 2^-32 is absorbed by the constants.
__device__ __forceinline__ uint32_t bconv_point(const int32_t* y, size_t stride, int n_in, const int32_t* m,
                                                uint32_t t, uint32_t tinv)
{
    const int64_t t31 = (int64_t)t << 31, t32 = (int64_t)t << 32;
    int64_t acc = 0;
    int s = 0;
    for (; s < n_in && s < 8; s++) acc += (int64_t)y[s * stride] * m[s];
    while (s < n_in) {
        acc = acc >= t31 ? acc - t32 : (acc < -t31 ? acc + t32 : acc);
        for (int e = 0; e < 4 && s < n_in; e++, s++) acc += (int64_t)y[s * stride] * m[s];
    }
    acc = acc >= t31 ? acc - t32 : (acc < -t31 ? acc + t32 : acc);
    return canon_signed(smr64(acc, t, tinv), t);
}

__device__ uint64_t dev_mulmod(uint64_t a, uint64_t b, uint64_t m) { return (a % m) * (b % m) % m; }
__device__ uint64_t dev_powmod(uint64_t a, uint64_t e, uint64_t m)
{
    uint64_t r = 1;
    a %= m;
    while (e) {
        if (e & 1) r = dev_mulmod(r, a, m);
        a = dev_mulmod(a, a, m);
        e >>= 1;
    }
    return r;
}

struct BconvIds {
    int8_t in[MAX_PRIMES];
    int8_t out[MAX_PRIMES];
    int n_in, n_out;
};

// constants: ws_c[s] = [Shat_s^-1]_s twisted; ws_m[t * n_in + s] = centred [Shat_s * 2^32]_t
// constants computed on the host, written to the workspace by one small
// launch (no host-to-device copy, so the call stays capture-safe)
constexpr int BCONV_FILL_MAX = 512;
struct BconvFill {
    int n_c, n_m;
    uint2 c[MAX_PRIMES];
    int32_t m[BCONV_FILL_MAX];
};
__global__ void k_bconv_fill(BconvFill F, uint2* ws_c, int32_t* ws_m)
{
    for (int i = threadIdx.x; i < F.n_m; i += blockDim.x) ws_m[i] = F.m[i];
    for (int i = threadIdx.x; i < F.n_c; i += blockDim.x) ws_c[i] = F.c[i];
}

__global__ void k_bconv_setup(const uint32_t* mods, const uint32_t* qinvs, BconvIds ids, uint2* ws_c, int32_t* ws_m)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;  // one thread per (target or -1 = inputs)
    if (t > ids.n_out) return;
    if (t == ids.n_out) {
        for (int s = 0; s < ids.n_in; s++) {
            const uint64_t qs = mods[ids.in[s]];
            uint64_t prod = 1;
            for (int r = 0; r < ids.n_in; r++)
                if (r != s) prod = dev_mulmod(prod, mods[ids.in[r]], qs);
            const uint64_t inv = dev_powmod(prod, qs - 2, qs);
            const uint32_t W = (uint32_t)((inv << 32) % qs);
            ws_c[s] = make_uint2(W, W * qinvs[ids.in[s]]);
        }
        return;
    }
    const uint64_t qt = mods[ids.out[t]];
    for (int s = 0; s < ids.n_in; s++) {
        uint64_t prod = 1;
        for (int r = 0; r < ids.n_in; r++)
            if (r != s) prod = dev_mulmod(prod, mods[ids.in[r]], qt);
        const uint64_t v = (prod << 32) % qt;
        ws_m[t * ids.n_in + s] = (int32_t)(2 * v < qt ? (int64_t)v : (int64_t)v - (int64_t)qt);
    }
}

__global__ void k_bconv_lift(const uint32_t* in, const uint32_t* mods, BconvIds ids, const uint2* ws_c, int32_t* y,
                             int log_n)
{
    const size_t n = (size_t)1 << log_n;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * ids.n_in) return;
    const int s = (int)(i >> log_n);
    const uint32_t q = mods[ids.in[s]];
    y[i] = lift(mulc(in[i], ws_c[s], q), q);
}

__global__ void k_bconv_matrix(const int32_t* y, const uint32_t* mods, const uint32_t* qinvs, BconvIds ids,
                               const int32_t* ws_m, uint32_t* out, int log_n)
{
    const size_t n = (size_t)1 << log_n;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * ids.n_out) return;
    const int t = (int)(i >> log_n);
    const size_t j = i & (n - 1);
    const int pid = ids.out[t];
    out[i] = bconv_point(y + j, n, ids.n_in, ws_m + t * ids.n_in, mods[pid], qinvs[pid]);
}

// ---------------------------------------------------------------------------
// launch helpers
// ---------------------------------------------------------------------------
static NttTables tables(const Ctx& c, bool inverse)
{
    return NttTables{inverse ? c.tw_inv : c.tw_fwd, inverse ? c.twq_inv : c.twq_fwd, c.mods, c.qinvs, c.log_n,
                     c.xcd_pair};
}

#define CKKS_DISPATCH_LOG1(log1, CALL)                  \
    switch (log1) {                                     \
    case 4: { constexpr int L1 = 4; CALL; } break;      \
    case 5: { constexpr int L1 = 5; CALL; } break;      \
    case 6: { constexpr int L1 = 6; CALL; } break;      \
    case 7: { constexpr int L1 = 7; CALL; } break;      \
    case 8: { constexpr int L1 = 8; CALL; } break;      \
    default: return set_error(-5, "unsupported ring degree"); \
    }

template <int L1, class MS, class Ld, class St>
static void fwd_cols(const Ctx& c, MS ms, int n, Ld ld, St st, hipStream_t s, int items_n = 1)
{
    if constexpr (L1 >= 5) {
        if (c.col_threads == 512) {
            CKKS_LAUNCH((k_fwd_cols<L1, MS, Ld, St, 512>), dim3(col_tiles<L1, 512>(), n, items_n), dim3(512), 0, s,
                        tables(c, false), ms, ld, st);
            return;
        }
    }
    if constexpr (L1 >= 7) {
        if (c.col_threads == 128) {
            CKKS_LAUNCH((k_fwd_cols<L1, MS, Ld, St, 128>), dim3(col_tiles<L1, 128>(), n, items_n), dim3(128), 0, s,
                        tables(c, false), ms, ld, st);
            return;
        }
    }
    CKKS_LAUNCH((k_fwd_cols<L1, MS, Ld, St>), dim3(col_tiles<L1>(), n, items_n), dim3(NTT_THREADS), 0, s,
                       tables(c, false), ms, ld, st);
}
// row passes: 16 residues per thread, or one wave per row (4); single
// operations (items_n == 1) and batched launches have knobs of their own
static int row_ept(const Ctx& c, int items_n) { return items_n > 1 ? c.rows_ept : c.rows_ept1; }
template <int L1, class MS, class Ld, class St>
static void fwd_rows(const Ctx& c, MS ms, int n, Ld ld, St st, hipStream_t s, int items_n = 1)
{
    if (row_ept(c, items_n) == 4)
        CKKS_LAUNCH((k_fwd_rows4<L1, MS, Ld, St>), dim3(row4_tiles<L1>(), n, items_n), dim3(NTT_THREADS), 0,
                           s, tables(c, false), ms, ld, st);
    else
        CKKS_LAUNCH((k_fwd_rows<L1, MS, Ld, St>), dim3(row_tiles<L1>(), n, items_n), dim3(NTT_THREADS), 0,
                           s, tables(c, false), ms, ld, st);
}
template <int L1, class MS, class Ld, class St>
static void inv_rows(const Ctx& c, MS ms, int n, Ld ld, St st, hipStream_t s, int items_n = 1)
{
    if (row_ept(c, items_n) == 4)
        CKKS_LAUNCH((k_inv_rows4<L1, MS, Ld, St>), dim3(row4_tiles<L1>(), n, items_n), dim3(NTT_THREADS), 0,
                           s, tables(c, true), ms, ld, st);
    else
        CKKS_LAUNCH((k_inv_rows<L1, MS, Ld, St>), dim3(row_tiles<L1>(), n, items_n), dim3(NTT_THREADS), 0,
                           s, tables(c, true), ms, ld, st);
}
template <int L1, class MS, class Ld, class St>
static void inv_cols(const Ctx& c, MS ms, int n, Ld ld, St st, hipStream_t s, int items_n = 1, int ct_force = 0,
                     bool c4 = false)
{
    if (c4) {  // 4 residues per thread (its BConv consumer must be k_bconv_ntt_cols4)
        CKKS_LAUNCH((k_inv_cols4<L1, MS, Ld, St>), dim3(Col4<L1>::TILES, n, items_n), dim3(NTT_THREADS), 0, s,
                    tables(c, true), ms, ld, st);
        return;
    }
    const int ct = ct_force ? ct_force : c.col_threads;  // a producer and its BConv consumer must agree
    if constexpr (L1 >= 5) {
        if (ct == 512) {
            CKKS_LAUNCH((k_inv_cols<L1, MS, Ld, St, 512>), dim3(col_tiles<L1, 512>(), n, items_n), dim3(512), 0, s,
                        tables(c, true), ms, ld, st);
            return;
        }
    }
    if constexpr (L1 >= 7) {
        if (ct == 128) {
            CKKS_LAUNCH((k_inv_cols<L1, MS, Ld, St, 128>), dim3(col_tiles<L1, 128>(), n, items_n), dim3(128), 0, s,
                        tables(c, true), ms, ld, st);
            return;
        }
    }
    CKKS_LAUNCH((k_inv_cols<L1, MS, Ld, St>), dim3(col_tiles<L1>(), n, items_n), dim3(NTT_THREADS), 0, s,
                       tables(c, true), ms, ld, st);
}

static int launched(const char* what) { return check_hip(hipGetLastError(), what); }
static MapByPtr ptr(const MapRef& m) { return MapByPtr{m.dev}; }
// key switching's column passes (INTT columns + BConv + NTT columns) with 4
// residues per thread: single operations and batched launches apart
static bool col4(const Ctx& c, int items_n) { return (items_n > 1 ? c.col_ept : c.col_ept1) == 4; }

template <int L1, int TPW, bool RS, class BS>
static void bconv_ntt(const Ctx& c, BS bs, int groups, int items_n, const int32_t* y, const int32_t* mat,
                      uint32_t* out, const BcRescale& X, size_t step, const BatchItem* items, hipStream_t s,
                      int ct_force = 0, bool c4 = false)
{
    if (c4) {
        CKKS_LAUNCH((k_bconv_ntt_cols4<L1, TPW, RS, BS>), dim3(Col4<L1>::TILES, groups, items_n), dim3(NTT_THREADS),
                    0, s, tables(c, false), bs, y, mat, out, X, step, items);
        return;
    }
    const int ct = ct_force ? ct_force : c.col_threads;
    if constexpr (L1 >= 5) {
        if (ct == 512) {
            CKKS_LAUNCH((k_bconv_ntt_cols<L1, TPW, 0, RS, BS, 512>), dim3(col_tiles<L1, 512>(), groups, items_n),
                        dim3(512), 0, s, tables(c, false), bs, y, mat, out, X, step, items);
            return;
        }
    }
    if constexpr (L1 >= 7) {
        if (ct == 128) {
            CKKS_LAUNCH((k_bconv_ntt_cols<L1, TPW, 0, RS, BS, 128>), dim3(col_tiles<L1, 128>(), groups, items_n),
                        dim3(128), 0, s, tables(c, false), bs, y, mat, out, X, step, items);
            return;
        }
    }
    CKKS_LAUNCH((k_bconv_ntt_cols<L1, TPW, 0, RS, BS>), dim3(col_tiles<L1>(), groups, items_n),
                       dim3(NTT_THREADS), 0, s, tables(c, false), bs, y, mat, out, X, step, items);
}

// one launch of the BConv + NTT column pass (map by pointer, or per level)
// tpw: targets per work-group the maps were built with (Ctx::tpw_up / tpw_dn)
template <bool RS, class BS>
static int launch_bconv_ntt(const Ctx& c, int tpw, BS bs, int groups, int items_n, const int32_t* y,
                            const int32_t* mat, uint32_t* out, const BcRescale& X, size_t step,
                            const BatchItem* items, hipStream_t s, int ct_force = 0, bool c4 = false)
{
    const int log1 = c.log_n - ROW_LOG;
    if (tpw == 1) { CKKS_DISPATCH_LOG1(log1, (bconv_ntt<L1, 1, RS>(c, bs, groups, items_n, y, mat, out, X, step, items, s, ct_force, c4))); }
    else if (tpw == 2) { CKKS_DISPATCH_LOG1(log1, (bconv_ntt<L1, 2, RS>(c, bs, groups, items_n, y, mat, out, X, step, items, s, ct_force, c4))); }
    else { CKKS_DISPATCH_LOG1(log1, (bconv_ntt<L1, 4, RS>(c, bs, groups, items_n, y, mat, out, X, step, items, s, ct_force, c4))); }
    return launched("bconv+ntt cols");
}

template <bool RS>
static int launch_bconv_list(const Ctx& c, int tpw, const std::vector<BcRef>& bs, const int32_t* y,
                             const int32_t* mat, uint32_t* out, const BcRescale& X, hipStream_t s, int ct_force = 0,
                             bool c4 = false)
{
    for (const BcRef& B : bs)
        if (int e = launch_bconv_ntt<RS>(c, tpw, BcByPtr{B.dev}, B.groups, 1, y, mat, out, X, 0, nullptr, s, ct_force,
                                         c4))
            return e;
    return 0;
}

// ---------------------------------------------------------------------------
// stand-alone NTT / INTT over a list of limbs (caller-chosen primes: maps by
// value)
// ---------------------------------------------------------------------------
int launch_ntt(const Ctx& c, bool inverse, uint32_t* data, const int32_t* pids, int n_limbs, hipStream_t s)
{
    const int log1 = c.log_n - ROW_LOG;
    for (int base = 0; base < n_limbs; base += MAX_LAUNCH_LIMBS) {
        const int n = n_limbs - base < MAX_LAUNCH_LIMBS ? n_limbs - base : MAX_LAUNCH_LIMBS;
        MapByVal M{};
        M.m.count = n;
        for (int l = 0; l < n; l++) {
            M.m.in_off[l] = M.m.out_off[l] = base + l;
            M.m.pid[l] = pids[base + l];
            M.m.cidx[l] = pids[base + l];
        }
        LdPlain ld{data, c.log_n};
        StPlain st{data, c.ninv, c.log_n};
        if (!inverse) {
            { KTimer t(c, "ntt_cols", s); CKKS_DISPATCH_LOG1(log1, (fwd_cols<L1>(c, M, n, ld, st, s))); }
            { KTimer t(c, "ntt_rows", s); CKKS_DISPATCH_LOG1(log1, (fwd_rows<L1>(c, M, n, ld, st, s))); }
        } else {
            { KTimer t(c, "intt_rows", s); CKKS_DISPATCH_LOG1(log1, (inv_rows<L1>(c, M, n, ld, st, s))); }
            { KTimer t(c, "intt_cols", s); CKKS_DISPATCH_LOG1(log1, (inv_cols<L1>(c, M, n, ld, st, s))); }
        }
        if (int e = launched("ntt")) return e;
    }
    return 0;
}

// ---------------------------------------------------------------------------
// stand-alone BConv (coefficient domain)
// ---------------------------------------------------------------------------
size_t bconv_ws_bytes(const Ctx& c, int n_in, int n_out)
{
    return 4096 + (size_t)n_in * n_out * 4 + ((size_t)n_in << c.log_n) * 4;
}

int launch_bconv(const Ctx& c, const uint32_t* in, const int32_t* in_ids, int n_in, uint32_t* out,
                 const int32_t* out_ids, int n_out, void* ws, hipStream_t s)
{
    BconvIds ids{};
    ids.n_in = n_in;
    ids.n_out = n_out;
    for (int i = 0; i < n_in; i++) ids.in[i] = (int8_t)in_ids[i];
    for (int i = 0; i < n_out; i++) ids.out[i] = (int8_t)out_ids[i];
    char* w = static_cast<char*>(ws);
    uint2* ws_c = reinterpret_cast<uint2*>(w);                        // <= 64 entries, 512 B
    int32_t* ws_m = reinterpret_cast<int32_t*>(w + 1024);              // n_out * n_in <= 3 KiB below 4096
    int32_t* y = reinterpret_cast<int32_t*>(w + 4096 + (size_t)n_in * n_out * 4);
    if (n_in * n_out * 4 > 4096 - 1024) ws_m = reinterpret_cast<int32_t*>(w + 4096), y = ws_m + n_in * n_out;
    KTimer tm(c, "bconv", s);
    if (n_in * n_out <= BCONV_FILL_MAX) {
        BconvFill F{};
        F.n_c = n_in, F.n_m = n_in * n_out;
        bconv_consts(c, in_ids, n_in, out_ids, n_out, F.c, F.m);
        CKKS_LAUNCH(k_bconv_fill, dim3(1), dim3(256), 0, s, F, ws_c, ws_m);
    } else {
        CKKS_LAUNCH(k_bconv_setup, dim3(1), dim3(128), 0, s, c.mods, c.qinvs, ids, ws_c, ws_m);
    }
    const size_t n = (size_t)1 << c.log_n;
    CKKS_LAUNCH(k_bconv_lift, dim3((unsigned)((n * n_in + 255) / 256)), dim3(256), 0, s, in, c.mods, ids, ws_c,
                       y, c.log_n);
    CKKS_LAUNCH(k_bconv_matrix, dim3((unsigned)((n * n_out + 255) / 256)), dim3(256), 0, s, y, c.mods, c.qinvs,
                       ids, ws_m, out, c.log_n);
    return launched("bconv");
}

// ---------------------------------------------------------------------------
// key switching: ModUp (INTT, BConv, NTT), KeyMult, ModDown
// ---------------------------------------------------------------------------
// workspace (units of N residues):
//   W0 [max(level, 2 (alpha+d))]      INTT row-pass output; later the P rows of ks (+ the d rows a
//                                     rescaling drops: 1, or a windowed level's dropped rows)
//   W1 [max(level, 2 (alpha+d))] int32  lifted ModUp input; later lifted ModDown input
//   W2 [max(beta (level+alpha), 2 level)]  ModUp column-pass output; later ModDown conv
//   W3 [2 level]                      ks on the Q rows
struct KsLayout {
    size_t w0, w1, w2, w3, total;  // offsets in residues
};
static KsLayout ks_layout(const Ctx& c, int level)
{
    const size_t n = (size_t)c.n;
    const int d = c.rs_drop_max(level);
    const size_t a = (size_t)(level > 2 * (c.n_p + d) ? level : 2 * (c.n_p + d));
    // ModUp rows of the largest level up to `level` (a window below the top
    // one can start inside a key digit and need one digit more)
    size_t up = 0;
    for (int l = 1; l <= level; l++)
        if (c.has_level(l) && (size_t)c.digits(l) * (l + c.n_p) > up) up = (size_t)c.digits(l) * (l + c.n_p);
    const size_t b = up > (size_t)2 * level ? up : (size_t)2 * level;
    KsLayout L;
    L.w0 = 0;
    L.w1 = L.w0 + a * n;
    L.w2 = L.w1 + a * n;
    L.w3 = L.w2 + b * n;
    L.total = L.w3 + (size_t)2 * level * n;
    return L;
}

size_t keyswitch_ws_bytes(const Ctx& c, int level) { return ks_layout(c, level).total * 4; }

template <int L1, Own OWN, Extra EX>
static void keymult(const Ctx& c, int max_level, int items_n, const KmArgs& A, hipStream_t s)
{
    if ((items_n == 1 ? c.km_ept1 : c.km_ept) == 4)
        CKKS_LAUNCH((k_keymult4<L1, OWN, EX>), dim3(row4_tiles<L1>(), max_level + c.n_p, items_n),
                    dim3(NTT_THREADS), 0, s, tables(c, false), tables(c, true), A);
    else
        CKKS_LAUNCH((k_keymult<L1, OWN, EX>), dim3(row_tiles<L1>(), max_level + c.n_p, items_n), dim3(NTT_THREADS),
                    0, s, tables(c, false), tables(c, true), A);
}

template <Own OWN, Extra EX>
static int keymult_dispatch(const Ctx& c, int max_level, int items_n, const KmArgs& A, hipStream_t s)
{
    CKKS_DISPATCH_LOG1(c.log_n - ROW_LOG, (keymult<L1, OWN, EX>(c, max_level, items_n, A, s)));
    return 0;
}

// Largest launch sizes over the context's levels in [lo, hi] (batched grids).
struct KsGrid {
    int up_rows = 0, up_cols = 0, up_bc = 0, dn_cols = 0, dn_bc = 0, dn_rows = 0;
};
static bool ks_grid(const Ctx& c, int lo, int hi, bool rescale, KsGrid& g)
{
    for (int level = lo; level <= hi; level++) {
        if (!c.has_level(level) || (rescale && c.windowed && !c.rr_below[level])) continue;
        const KsPlan& P = c.ks_plan[rescale ? 1 : 0][level];
        if (P.up_bc.size() != 1 || P.dn_bc.size() != 1) return false;
        g.up_rows = std::max(g.up_rows, P.up_rows.n);
        g.up_cols = std::max(g.up_cols, P.up_cols.n);
        g.up_bc = std::max(g.up_bc, P.up_bc[0].groups);
        g.dn_cols = std::max(g.dn_cols, P.dn_cols.n);
        g.dn_bc = std::max(g.dn_bc, P.dn_bc[0].groups);
        g.dn_rows = std::max(g.dn_rows, P.dn_rows.n);
    }
    return true;
}

// Where the phases of a key switch find their maps, workspace and items.
// Single operation: this level's plan, z = 1.  Batched: the per-level
// directory, z = items, workspace slices ws_step apart.
struct KsRun {
    const Ctx* c;
    const KsPlan* P = nullptr;  // single
    const KsDir* D = nullptr;   // batched
    const BatchItem* items = nullptr;
    int zn = 1, lo = 1, hi = 1, nk = 1, ns = 1;
    KsGrid g;
    size_t wst = 0;
    uint32_t* w0;
    int32_t* w1;
    uint32_t* w2;
    uint32_t* w3;
};

#define KS_MAP(R, field, CALL)                                      \
    do {                                                            \
        if ((R).D) {                                                \
            MapDir ms{(R).D->field, (R).items, (R).lo, (R).hi, (R).nk, (R).ns}; \
            CALL;                                                   \
        } else {                                                    \
            MapByPtr ms{(R).P->field.dev};                          \
            CALL;                                                   \
        }                                                           \
    } while (0)

static KsRun ks_run(const Ctx& c, void* ws, int top)
{
    KsRun R;
    R.c = &c;
    const KsLayout L = ks_layout(c, top);
    uint32_t* W = static_cast<uint32_t*>(ws);
    R.w0 = W + L.w0;
    R.w1 = reinterpret_cast<int32_t*>(W + L.w1);
    R.w2 = W + L.w2;
    R.w3 = W + L.w3;
    return R;
}

// ModUp: INTT (row and column pass, with the prologue of `own`), BConv +
// NTT column pass.  Leaves the lifted digits in w1 and the new rows' column
// pass in w2.
static int modup_phase(const KsRun& R, Own own, const KsIn& in, size_t s0, size_t s1, hipStream_t s)
{
    const Ctx& c = *R.c;
    const int log1 = c.log_n - ROW_LOG;
    const bool c4 = col4(c, R.zn);
    {
        StPlain st{R.w0, nullptr, c.log_n, R.wst};
        const uint32_t gal = (uint32_t)in.galois;
        KTimer t(c, "modup_intt_rows", s);
        switch (own) {
        case Own::Tensor: { LdOwn<Own::Tensor> ld{in.a0, in.a1, gal, c.log_n, s0, s1, R.items}; KS_MAP(R, up_rows, CKKS_DISPATCH_LOG1(log1, (inv_rows<L1>(c, ms, R.g.up_rows, ld, st, s, R.zn)))); } break;
        case Own::Gather: { LdOwn<Own::Gather> ld{in.a0, in.a1, gal, c.log_n, s0, s1, R.items}; KS_MAP(R, up_rows, CKKS_DISPATCH_LOG1(log1, (inv_rows<L1>(c, ms, R.g.up_rows, ld, st, s, R.zn)))); } break;
        default:          { LdOwn<Own::Plain> ld{in.a0, in.a1, gal, c.log_n, s0, s1, R.items};  KS_MAP(R, up_rows, CKKS_DISPATCH_LOG1(log1, (inv_rows<L1>(c, ms, R.g.up_rows, ld, st, s, R.zn)))); } break;
        }
        if (int e = launched("modup intt rows")) return e;
    }
    {
        LdPlain ld{R.w0, c.log_n, R.wst};
        StLift st{R.w1, own == Own::Tensor ? c.up_c_r : c.up_c, c.log_n, R.wst};
        KTimer t(c, "modup_intt_cols", s);
        KS_MAP(R, up_cols, CKKS_DISPATCH_LOG1(log1, (inv_cols<L1>(c, ms, R.g.up_cols, ld, st, s, R.zn, 0, c4))));
        if (int e = launched("modup intt cols")) return e;
    }
    {
        KTimer t(c, "modup_bconv_ntt_cols", s);
        int e;
        if (R.D) e = launch_bconv_ntt<false>(c, c.tpw_up, BcDir{R.D->up_bc, R.items, R.lo, R.hi, R.nk, R.ns}, R.g.up_bc, R.zn, R.w1, c.up_mat, R.w2, BcRescale{}, R.wst, R.items, s, 0, c4);
        else e = launch_bconv_list<false>(c, c.tpw_up, R.P->up_bc, R.w1, c.up_mat, R.w2, BcRescale{}, s, 0, c4);
        if (e) return e;
    }
    return 0;
}

// ModDown: INTT column pass of the P rows (+ row l-1 when rescaling), BConv
// P -> Q + NTT column pass, NTT row pass + combine into out0 / out1.
static int moddown_phase(const KsRun& R, int level, bool rescale, uint32_t* out0, uint32_t* out1, size_t out_step,
                         hipStream_t s)
{
    const Ctx& c = *R.c;
    const int log1 = c.log_n - ROW_LOG;
    const bool rr = rescale && c.windowed;  // merged ModDown + rational rescaling
    const bool c4 = col4(c, R.zn);
    {
        LdPlain ld{R.w0, c.log_n, R.wst};
        StLift st{R.w1, rr ? c.rr_c : c.dn_c, c.log_n, R.wst};
        KTimer t(c, "moddown_intt_cols", s);
        KS_MAP(R, dn_cols, CKKS_DISPATCH_LOG1(log1, (inv_cols<L1>(c, ms, R.g.dn_cols, ld, st, s, R.zn, 0, c4))));
        if (int e = launched("moddown intt cols")) return e;
    }
    {
        KTimer t(c, "moddown_bconv_ntt_cols", s);
        const BcRescale X{c.rs_mlast, c.rs_pr, c.n_p, level};
        int e;
        if (R.D) {
            const BcDir bd{R.D->dn_bc, R.items, R.lo, R.hi, R.nk, R.ns};
            if (rr) e = launch_bconv_ntt<false>(c, c.tpw_dn, bd, R.g.dn_bc, R.zn, R.w1, c.rr_mat, R.w2, X, R.wst, R.items, s, 0, c4);
            else if (rescale) e = launch_bconv_ntt<true>(c, c.tpw_dn, bd, R.g.dn_bc, R.zn, R.w1, c.dn_mat, R.w2, X, R.wst, R.items, s, 0, c4);
            else e = launch_bconv_ntt<false>(c, c.tpw_dn, bd, R.g.dn_bc, R.zn, R.w1, c.dn_mat, R.w2, X, R.wst, R.items, s, 0, c4);
        } else {
            if (rr) e = launch_bconv_list<false>(c, c.tpw_dn, R.P->dn_bc, R.w1, c.rr_mat, R.w2, X, s, 0, c4);
            else if (rescale) e = launch_bconv_list<true>(c, c.tpw_dn, R.P->dn_bc, R.w1, c.dn_mat, R.w2, X, s, 0, c4);
            else e = launch_bconv_list<false>(c, c.tpw_dn, R.P->dn_bc, R.w1, c.dn_mat, R.w2, X, s, 0, c4);
        }
        if (e) return e;
    }
    {
        LdPlain ld{R.w2, c.log_n, R.wst};
        StCombine st{out0, out1, R.w3, rr ? c.rr_fin : rescale ? c.rs_fin : c.dn_pinv, c.log_n, out_step, R.wst};
        KTimer t(c, "moddown_ntt_rows_combine", s);
        KS_MAP(R, dn_rows, CKKS_DISPATCH_LOG1(log1, (fwd_rows<L1>(c, ms, R.g.dn_rows, ld, st, s, R.zn))));
        if (int e = launched("moddown ntt rows")) return e;
    }
    return 0;
}

static int keymult_launch(const Ctx& c, Own own, Extra extra, int top, int zn, const KmArgs& A, hipStream_t s)
{
    KTimer t(c, "keymult", s);
    int e;
    if (own == Own::Tensor && extra == Extra::HMult) e = keymult_dispatch<Own::Tensor, Extra::HMult>(c, top, zn, A, s);
    else if (own == Own::Plain && extra == Extra::None) e = keymult_dispatch<Own::Plain, Extra::None>(c, top, zn, A, s);
    else if (own == Own::Gather && extra == Extra::HRot) e = keymult_dispatch<Own::Gather, Extra::HRot>(c, top, zn, A, s);
    else if (own == Own::Hoisted && extra == Extra::HRot) e = keymult_dispatch<Own::Hoisted, Extra::HRot>(c, top, zn, A, s);
    else return set_error(-1, "unsupported key-switch variant");
    if (e) return e;
    return launched("keymult");
}

static KmArgs km_args(const Ctx& c, const KsRun& R, const KsIn& in, const uint32_t* evk, int level, bool rescale)
{
    KmArgs A{};
    A.up = R.w2;
    A.evk = evk;
    A.b0 = in.b0;
    A.a0 = in.a0;
    A.b1 = in.b1;
    A.a1 = in.a1;
    A.ks_q = R.w3;
    A.ks_p = R.w0;
    A.p_mod_q = c.p_mod_q;
    A.rinv = c.rinv;
    A.p_r2 = c.p_r2;
    A.r1 = c.r1;
    A.galois = (uint32_t)in.galois;
    A.level = level;
    A.n_q = c.n_q;
    A.n_p = c.n_p;
    A.base = c.wbase[level];  // batched launches run on prefix contexts only (base 0 at every level)
    A.rs = rescale ? c.rs_drop(level) : 0;
    A.dlo = c.windowed ? c.rr_dlo[level] : 0;
    A.dhi = c.windowed ? c.rr_dhi[level] : -1;
    A.lv = nullptr;  // set for batched launches on a windowed context
    A.lo_level = R.lo;
    A.n_keys = R.nk;
    A.n_src = R.ns;
    return A;
}

// Shared sequence of a single (b == nullptr) or batched key switch.
static int keyswitch_seq(const Ctx& c, Own own, Extra extra, const KsIn& in, int level, const KsBatch* b,
                         const uint32_t* evk, uint32_t* out0, uint32_t* out1, void* ws, hipStream_t s, bool rescale)
{
    const int rsi = rescale ? 1 : 0;
    const int top = b ? b->max_level : level;  // layout and grids are sized for this level
    KsRun R = ks_run(c, ws, top);
    if (b) {
        if (!ks_grid(c, rescale && !c.windowed ? 2 : 1, top, rescale, R.g) || !c.ks_dir[rsi].up_rows)
            return set_error(-5, "batched key switching is not available at these levels");
        R.D = &c.ks_dir[rsi];
        R.items = b->items;
        R.zn = b->n;
        R.lo = rescale && !c.windowed ? 2 : 1;
        R.hi = top;
        R.nk = b->n_keys;
        R.ns = b->n_src;
        R.wst = b->ws_step;
    } else {
        R.P = &c.ks_plan[rsi][level];
        if (!R.P->up_rows.dev) return set_error(-5, "no launch plan for this level");
        R.g.up_rows = R.P->up_rows.n, R.g.up_cols = R.P->up_cols.n;
        R.g.dn_cols = R.P->dn_cols.n, R.g.dn_rows = R.P->dn_rows.n;
    }
    if (int e = modup_phase(R, own, in, b ? b->in_step : 0, b ? b->in2_step : 0, s)) return e;
    KmArgs A = km_args(c, R, in, evk, top, rescale);
    if (b) {
        A.items = b->items;
        A.in_step = b->in_step, A.in2_step = b->in2_step, A.key_step = b->key_step;
        A.ws_step = A.up_step = b->ws_step;
        if (c.windowed) A.lv = c.lv_tab;
    }
    if (int e = keymult_launch(c, own, extra, top, R.zn, A, s)) return e;
    return moddown_phase(R, level, rescale, out0, out1, b ? b->out_step : 0, s);
}

// Hoisted HRot: one ModUp of a (materialised in the evaluation domain),
// then KeyMult with the automorphism gathered on load and ModDown for every
// rotation at once (grid.z = rotation).  Workspace: one key-switch layout
// for the shared ModUp, then one per rotation.
int launch_hrot_hoisted(const Ctx& c, const uint32_t* b_in, const uint32_t* a_in, int level, int n_rot,
                        const BatchItem* items, const uint32_t* keys, int n_keys, size_t key_step, uint32_t* outs,
                        void* ws, hipStream_t s)
{
    const int log1 = c.log_n - ROW_LOG;
    const KsPlan& P = c.ks_plan[0][level];
    if (!P.up_rows.dev || !P.up_nrows.dev || !c.ks_dir[0].dn_bc) return set_error(-5, "no launch plan for this level");
    const size_t slice = keyswitch_ws_bytes(c, level) / 4;
    KsRun U = ks_run(c, ws, level);  // shared ModUp
    U.P = &P;
    U.g.up_rows = P.up_rows.n, U.g.up_cols = P.up_cols.n;
    KsIn in;
    in.b0 = b_in;
    in.a0 = a_in;
    if (int e = modup_phase(U, Own::Plain, in, 0, 0, s)) return e;
    {  // complete the ModUp rows in the evaluation domain (row pass in place)
        LdPlain ld{U.w2, c.log_n};
        StPlain st{U.w2, nullptr, c.log_n};
        KTimer t(c, "modup_ntt_rows", s);
        CKKS_DISPATCH_LOG1(log1, (fwd_rows<L1>(c, MapByPtr{P.up_nrows.dev}, P.up_nrows.n, ld, st, s)));
        if (int e = launched("modup ntt rows")) return e;
    }
    KsRun R = ks_run(c, static_cast<uint32_t*>(ws) + slice, level);  // rotation 0's slice
    R.D = &c.ks_dir[0];
    R.items = items;
    R.zn = n_rot;
    R.lo = R.hi = level;
    R.nk = n_keys;
    R.ns = 0;  // every rotation reads the one input; item slots are not used
    R.wst = slice;
    if (!ks_grid(c, level, level, false, R.g)) return set_error(-5, "no launch plan for this level");
    KmArgs A = km_args(c, R, in, keys, level, false);
    A.up = U.w2;
    A.items = items;
    A.key_step = key_step;
    A.ws_step = slice;
    A.up_step = 0;
    if (int e = keymult_launch(c, Own::Hoisted, Extra::HRot, level, n_rot, A, s)) return e;
    const size_t out_step = 2 * (size_t)level * c.n;
    return moddown_phase(R, level, false, outs, outs + (size_t)level * c.n, out_step, s);
}

template <int L1>
static void keymult_sum(const Ctx& c, int level, const KmArgs& A, const uint32_t* pts, size_t pt_step, int n_rot,
                        hipStream_t s)
{
    CKKS_LAUNCH((k_keymult_sum<L1>), dim3(row_tiles<L1>(), level + c.n_p, 1), dim3(NTT_THREADS), 0, s,
                tables(c, false), tables(c, true), A, pts, pt_step, n_rot, (const uint2*)c.r1);
}

// Sum of plaintext-weighted rotations: the hoisted ModUp (as above), one
// KeyMult pass over every rotation, one ModDown.  Workspace: the shared
// ModUp layout, then one key-switch layout.
int launch_hrot_sum_hoisted(const Ctx& c, const uint32_t* b_in, const uint32_t* a_in, int level, int n_rot,
                            const BatchItem* items, const uint32_t* keys, int n_keys, size_t key_step,
                            const uint32_t* pts, size_t pt_step, uint32_t* out, void* ws, hipStream_t s)
{
    const int log1 = c.log_n - ROW_LOG;
    const KsPlan& P = c.ks_plan[0][level];
    if (!P.up_rows.dev || !P.up_nrows.dev) return set_error(-5, "no launch plan for this level");
    const size_t slice = keyswitch_ws_bytes(c, level) / 4;
    KsRun U = ks_run(c, ws, level);
    U.P = &P;
    U.g.up_rows = P.up_rows.n, U.g.up_cols = P.up_cols.n;
    KsIn in;
    in.b0 = b_in;
    in.a0 = a_in;
    if (int e = modup_phase(U, Own::Plain, in, 0, 0, s)) return e;
    {
        LdPlain ld{U.w2, c.log_n};
        StPlain st{U.w2, nullptr, c.log_n};
        KTimer t(c, "modup_ntt_rows", s);
        CKKS_DISPATCH_LOG1(log1, (fwd_rows<L1>(c, MapByPtr{P.up_nrows.dev}, P.up_nrows.n, ld, st, s)));
        if (int e = launched("modup ntt rows")) return e;
    }
    KsRun R = ks_run(c, static_cast<uint32_t*>(ws) + slice, level);
    R.P = &P;
    R.g.up_rows = P.up_rows.n, R.g.up_cols = P.up_cols.n;
    R.g.dn_cols = P.dn_cols.n, R.g.dn_rows = P.dn_rows.n;
    R.nk = n_keys;
    KmArgs A = km_args(c, R, in, keys, level, false);
    A.up = U.w2;
    A.items = items;
    A.key_step = key_step;
    {
        KTimer t(c, "keymult_sum", s);
        CKKS_DISPATCH_LOG1(log1, (keymult_sum<L1>(c, level, A, pts, pt_step, n_rot, s)));
        if (int e = launched("keymult sum")) return e;
    }
    return moddown_phase(R, level, false, out, out + (size_t)level * c.n, 0, s);
}

int launch_keyswitch(const Ctx& c, Own own, Extra extra, const KsIn& in, int level, const uint32_t* evk,
                     uint32_t* out0, uint32_t* out1, void* ws, hipStream_t s, bool rescale)
{
    if (rescale && c.rs_out(level) < 1) return set_error(-1, "no level below this one to rescale to");
    return keyswitch_seq(c, own, extra, in, level, nullptr, evk, out0, out1, ws, s, rescale);
}

int launch_keyswitch_batch(const Ctx& c, Own own, Extra extra, const KsIn& in, const KsBatch& b,
                           const uint32_t* evk, uint32_t* out0, uint32_t* out1, void* ws, hipStream_t s,
                           bool rescale)
{
    if (b.n < 1 || b.n > 65535) return set_error(-1, "batch size out of range");
    return keyswitch_seq(c, own, extra, in, b.max_level, &b, evk, out0, out1, ws, s, rescale);
}

// ---------------------------------------------------------------------------
// rescale: t = lift(INTT(c_{l-1})), c'_i = (c_i - NTT([t]_{q_i})) q_{l-1}^-1
// ---------------------------------------------------------------------------
size_t rescale_ws_bytes(const Ctx& c) { return ((size_t)4 + 2 * (size_t)c.n_q) * (size_t)c.n * 4; }

int launch_rescale(const Ctx& c, const uint32_t* in, int level_in, uint32_t* out, void* ws, hipStream_t s)
{
    const int log1 = c.log_n - ROW_LOG;
    const RsPlan& P = c.rs_plan[level_in];
    if (!P.rows.dev) return set_error(-5, "no launch plan for this level");
    uint32_t* W = static_cast<uint32_t*>(ws);
    uint32_t* w0 = W;                                               // [2] INTT row pass of the last limbs
    int32_t* w1 = reinterpret_cast<int32_t*>(W + 2 * (size_t)c.n);  // [2] lifted t
    uint32_t* w2 = W + 4 * (size_t)c.n;                             // [2 (l-1)] NTT column pass of [t]_{q_i}
    {
        LdPlain ld{in, c.log_n};
        StPlain st{w0, nullptr, c.log_n};
        { KTimer t(c, "rescale_intt_rows", s); CKKS_DISPATCH_LOG1(log1, (inv_rows<L1>(c, ptr(P.rows), 2, ld, st, s))); }
        LdPlain ld2{w0, c.log_n};
        StLift st2{w1, c.ninv, c.log_n};
        { KTimer t(c, "rescale_intt_cols", s); CKKS_DISPATCH_LOG1(log1, (inv_cols<L1>(c, ptr(P.cols), 2, ld2, st2, s))); }
        if (int e = launched("rescale intt")) return e;
    }
    {
        LdCentred ld{w1, c.log_n};
        StPlain st{w2, nullptr, c.log_n};
        KTimer t(c, "rescale_ntt_cols", s);
        CKKS_DISPATCH_LOG1(log1, (fwd_cols<L1>(c, ptr(P.ncols), P.ncols.n, ld, st, s)));
        if (int e = launched("rescale ntt cols")) return e;
    }
    {
        LdPlain ld{w2, c.log_n};
        StCombine st{out, out, in, c.rs_qinv, c.log_n};
        KTimer t(c, "rescale_ntt_rows_combine", s);
        CKKS_DISPATCH_LOG1(log1, (fwd_rows<L1>(c, ptr(P.nrows), P.nrows.n, ld, st, s)));
        if (int e = launched("rescale ntt rows")) return e;
    }
    return 0;
}

// ---------------------------------------------------------------------------
// launch plans: every map an internal launch needs, built once per context
// ---------------------------------------------------------------------------
namespace {

struct Blob {
    std::vector<char> bytes;
    size_t add(const void* p, size_t n)
    {
        const size_t off = (bytes.size() + 255) & ~(size_t)255;
        bytes.resize(off + n);
        std::memcpy(bytes.data() + off, p, n);
        return off;
    }
};

// offsets are stored in the pointer fields until the blob is uploaded
template <class T>
T* as_off(size_t off) { return reinterpret_cast<T*>(off); }
template <class T>
void rebase(const T*& p, char* base) { p = reinterpret_cast<const T*>(base + reinterpret_cast<size_t>(p)); }

MapRef add_map(Blob& b, LaunchMap m, int n)
{
    m.count = n;
    return MapRef{as_off<const LaunchMap>(b.add(&m, sizeof m)), n};
}

// groups of at most tpw targets sharing input rows; one BcMap per launch
struct BcBuilder {
    Blob& blob;
    int tpw;
    std::vector<BcRef>& out;
    BcMap B{};
    int groups = 0, targets = 0, n_in_max = 0;
    void flush()
    {
        if (!groups) return;
        B.groups = groups;
        out.push_back(BcRef{as_off<const BcMap>(blob.add(&B, sizeof B)), groups, n_in_max});
        B = BcMap{};
        groups = targets = n_in_max = 0;
    }
    void add(int in_off, int n_in, int n, const int32_t* mat_off, const int32_t* out_off, const int8_t* pid)
    {
        for (int i = 0; i < n; i += tpw) {
            const int cnt = n - i < tpw ? n - i : tpw;
            if (groups == MAX_BC_GROUPS || targets + cnt > MAX_LAUNCH_LIMBS) flush();
            B.in_off[groups] = in_off;
            B.n_in[groups] = n_in;
            B.first[groups] = targets;
            B.n_tg[groups] = cnt;
            for (int k = 0; k < cnt; k++) {
                B.mat_off[targets + k] = mat_off[i + k];
                B.out_off[targets + k] = out_off[i + k];
                B.pid[targets + k] = pid[i + k];
            }
            groups++;
            targets += cnt;
            n_in_max = n_in > n_in_max ? n_in : n_in_max;
        }
    }
};

void build_ks_plan(const Ctx& c, Blob& b, int level, bool rescale, KsPlan& P)
{
    const int alpha = c.n_p, beta = c.digits(level), rows = level + alpha;
    const int rs = rescale ? c.rs_drop(level) : 0, pst = alpha + rs, out_rows = rescale ? c.rs_out(level) : level;
    const int wb = c.wbase[level];  // prime id of the level's first limb
    // merged ModDown + rational rescaling (windowed context): the rows after
    // P in ks_p are the dropped window rows in row order; outputs are the
    // window below, starting at prime id ob
    const bool rr = rescale && c.windowed;
    const int ob = rr ? c.wbase[out_rows] : wb;
    int dpid[MAX_PRIMES] = {};
    for (int r = 0, k = 0; rr && r < level; r++)
        if (r < c.rr_dlo[level] || r >= c.rr_dhi[level]) dpid[k++] = wb + r;
    {  // ModUp INTT passes over the level limbs
        LaunchMap M{};
        for (int i = 0; i < level; i++) {
            M.in_off[i] = M.out_off[i] = i;
            M.pid[i] = (wb + i);
            M.cidx[i] = (level * c.n_q + wb + i);
        }
        P.up_rows = add_map(b, M, level);
        P.up_cols = add_map(b, M, level);
    }
    {  // ModUp rows other than each digit's own, for the evaluation-domain row pass (hoisted HRot)
        LaunchMap M{};
        int n = 0;
        for (int j = 0; j < beta; j++) {
            const int lo = c.digit_lo(j, level), hi = c.digit_hi(j, level);
            for (int r = 0; r < rows; r++) {
                if (r >= lo && r < hi) continue;
                if (n < MAX_LAUNCH_LIMBS) {
                    M.in_off[n] = M.out_off[n] = j * rows + r;
                    M.pid[n] = c.row_pid(r, level);
                }
                n++;
            }
        }
        if (n <= MAX_LAUNCH_LIMBS) P.up_nrows = add_map(b, M, n);
    }
    {  // ModUp BConv: digit j -> every other row
        BcBuilder bb{b, c.tpw_up, P.up_bc};
        int32_t mo[2 * MAX_PRIMES], oo[2 * MAX_PRIMES];
        int8_t pd[2 * MAX_PRIMES];
        for (int j = 0; j < beta; j++) {
            const int lo = c.digit_lo(j, level), hi = c.digit_hi(j, level);
            int n = 0;
            for (int r = 0; r < rows; r++) {
                if (r >= lo && r < hi) continue;
                const int pid = c.row_pid(r, level);
                mo[n] = ((level * c.dnum + c.key_digit(j, level)) * c.n_primes + pid) * c.n_p;
                oo[n] = j * rows + r;
                pd[n] = (int8_t)pid;
                n++;
            }
            bb.add(lo, hi - lo, n, mo, oo, pd);
        }
        bb.flush();
    }
    {  // ModDown INTT column pass (P rows, and row q_{l-1} when rescaling)
        LaunchMap M{};
        for (int poly = 0; poly < 2; poly++)
            for (int k = 0; k < pst; k++) {
                const int l = poly * pst + k;
                M.in_off[l] = M.out_off[l] = l;
                if (rr) {
                    M.pid[l] = (k < alpha ? c.n_q + k : dpid[k - alpha]);
                    M.cidx[l] = (c.rr_c_off[level] + k);
                } else {
                    M.pid[l] = (k < alpha ? c.n_q + k : level - 1);
                    M.cidx[l] = (k < alpha ? k : c.n_p + level - 1);
                }
            }
        P.dn_cols = add_map(b, M, 2 * pst);
    }
    {  // ModDown BConv P -> Q (merged: P u dropped rows -> the window below)
        BcBuilder bb{b, c.tpw_dn, P.dn_bc};
        int32_t mo[MAX_PRIMES], oo[MAX_PRIMES];
        int8_t pd[MAX_PRIMES];
        for (int poly = 0; poly < 2; poly++) {
            for (int i = 0; i < out_rows; i++) {
                mo[i] = rr ? c.rr_mat_off[level] + i * pst : (wb + i) * c.n_p;
                oo[i] = poly * out_rows + i;
                pd[i] = (int8_t)(ob + i);
            }
            bb.add(poly * pst, rr ? pst : alpha, out_rows, mo, oo, pd);
        }
        bb.flush();
    }
    {  // ModDown NTT row pass + combine: the two polynomials' limbs of a prime
        // are neighbours in the map (launch limbs 2i, 2i + 1), so the work-groups
        // that read a row's twiddles twice run together on one XCD (grid.x is a
        // multiple of 8) and the second read hits its L2
        LaunchMap M{};
        for (int poly = 0; poly < 2; poly++)
            for (int i = 0; i < out_rows; i++) {
                const int l = 2 * i + poly;
                const int r = ob + i - wb;  // the output prime's row in ks_q, if the window has it
                M.in_off[l] = poly * out_rows + i;
                M.sub_off[l] = r >= 0 && r < level ? poly * level + r : -1;
                M.out_off[l] = i;
                M.grp[l] = poly;
                M.pid[l] = (ob + i);
                M.cidx[l] = (rr ? c.rr_fin_off[level] + i : rescale ? level * c.n_q + i : wb + i);
            }
        P.dn_rows = add_map(b, M, 2 * out_rows);
    }
}

void build_rs_plan(const Ctx& c, Blob& b, int level, RsPlan& P)
{
    const int lo = level - 1;
    LaunchMap M{};
    for (int poly = 0; poly < 2; poly++) {
        M.in_off[poly] = poly * level + lo;
        M.out_off[poly] = poly;
        M.pid[poly] = lo;
        M.cidx[poly] = lo;
    }
    P.rows = add_map(b, M, 2);
    M.in_off[0] = 0, M.in_off[1] = 1;
    P.cols = add_map(b, M, 2);
    LaunchMap N{};
    for (int poly = 0; poly < 2; poly++)
        for (int i = 0; i < lo; i++) {
            const int l = poly * lo + i;
            N.in_off[l] = poly;
            N.out_off[l] = l;
            N.pid[l] = i;
        }
    P.ncols = add_map(b, N, 2 * lo);
    LaunchMap R{};
    for (int poly = 0; poly < 2; poly++)
        for (int i = 0; i < lo; i++) {
            const int l = poly * lo + i;
            R.in_off[l] = l;
            R.sub_off[l] = poly * level + i;
            R.out_off[l] = poly * lo + i;
            R.pid[l] = i;
            R.cidx[l] = (level * c.n_q + i);
        }
    P.nrows = add_map(b, R, 2 * lo);
}

// stand-alone rational rescaling from the window at `level` to the window
// below: INTT of the dropped rows (both halves), BConv to the output primes +
// NTT column pass, NTT row pass + combine with the kept input rows
void build_rr_plan(const Ctx& c, Blob& b, int level, RrPlan& P)
{
    const int wb = c.wbase[level], below = c.rr_below[level], ob = c.wbase[below];
    const int nd = c.rr_drop(level);
    int dr[MAX_PRIMES] = {};
    for (int r = 0, k = 0; r < level; r++)
        if (r < c.rr_dlo[level] || r >= c.rr_dhi[level]) dr[k++] = r;
    LaunchMap M{};
    for (int poly = 0; poly < 2; poly++)
        for (int k = 0; k < nd; k++) {
            const int l = poly * nd + k;
            M.in_off[l] = poly * level + dr[k];
            M.out_off[l] = l;
            M.pid[l] = (wb + dr[k]);
            M.cidx[l] = (c.rr2_c_off[level] + k);
        }
    P.rows = add_map(b, M, 2 * nd);
    for (int l = 0; l < 2 * nd; l++) M.in_off[l] = l;
    P.cols = add_map(b, M, 2 * nd);
    // one target per work-group: a few dropped rows convert to a window's
    // worth of targets, and the launch needs the work-groups more than the
    // shared input loads
    BcBuilder bb{b, 1, P.bc};
    int32_t mo[MAX_PRIMES], oo[MAX_PRIMES];
    int8_t pd[MAX_PRIMES];
    for (int poly = 0; poly < 2; poly++) {
        for (int o = 0; o < below; o++) {
            mo[o] = c.rr2_mat_off[level] + o * nd;
            oo[o] = poly * below + o;
            pd[o] = (int8_t)(ob + o);
        }
        bb.add(poly * nd, nd, below, mo, oo, pd);
    }
    bb.flush();
    LaunchMap R{};
    for (int poly = 0; poly < 2; poly++)
        for (int o = 0; o < below; o++) {
            const int l = poly * below + o, r = ob + o - wb;
            R.in_off[l] = l;
            R.sub_off[l] = r >= 0 && r < level ? poly * level + r : -1;
            R.out_off[l] = o;
            R.grp[l] = poly;
            R.pid[l] = (ob + o);
            R.cidx[l] = (c.rr2_fin_off[level] + o);
        }
    P.nrows = add_map(b, R, 2 * below);
}

}  // namespace

// The four-pass rescaling runs a few rows: its column passes use the
// narrowest tiles (twice the work-groups; applied where N >= 2^15, both
// the lifting INTT and the BConv that reads its tile layout).
constexpr int RR_COL_THREADS = 128;

int launch_rescale_rational_window(const Ctx& c, int level, const uint32_t* ct, uint32_t* out, void* ws,
                                   hipStream_t s)
{
    const RrPlan& P = c.rr_plan[level];
    if (!P.rows.dev) return set_error(-5, "no rational rescaling plan for this level");
    const int log1 = c.log_n - ROW_LOG, nd = c.rr_drop(level), below = c.rr_below[level];
    const size_t n = c.n;
    uint32_t* w0 = static_cast<uint32_t*>(ws);
    int32_t* w1 = reinterpret_cast<int32_t*>(w0 + 2 * (size_t)nd * n);
    uint32_t* w2 = reinterpret_cast<uint32_t*>(w1 + 2 * (size_t)nd * n);
    {
        LdPlain ld{ct, c.log_n};
        StPlain st{w0, nullptr, c.log_n};
        KTimer t(c, "rr_intt_rows", s);
        CKKS_DISPATCH_LOG1(log1, (inv_rows<L1>(c, MapByPtr{P.rows.dev}, P.rows.n, ld, st, s)));
        if (int e = launched("rational rescale intt rows")) return e;
    }
    {
        LdPlain ld{w0, c.log_n};
        StLift st{w1, c.rr2_c, c.log_n};
        KTimer t(c, "rr_intt_cols", s);
        CKKS_DISPATCH_LOG1(log1, (inv_cols<L1>(c, MapByPtr{P.cols.dev}, P.cols.n, ld, st, s, 1, RR_COL_THREADS)));
        if (int e = launched("rational rescale intt cols")) return e;
    }
    {
        KTimer t(c, "rr_bconv_ntt_cols", s);
        if (int e = launch_bconv_list<false>(c, 1, P.bc, w1, c.rr2_mat, w2, BcRescale{}, s, RR_COL_THREADS))
            return e;
    }
    {
        LdPlain ld{w2, c.log_n};
        StCombine st{out, out + (size_t)below * n, ct, c.rr2_fin, c.log_n};
        KTimer t(c, "rr_ntt_rows_combine", s);
        CKKS_DISPATCH_LOG1(log1, (fwd_rows<L1>(c, MapByPtr{P.nrows.dev}, P.nrows.n, ld, st, s)));
        if (int e = launched("rational rescale ntt rows")) return e;
    }
    return 0;
}

// Rebuild the launch plans for new tuning knobs (the caller has drained
// every stream that uses the context).
int retune(Ctx& c, int tpw_up, int tpw_dn, int xcd_pair, int rows_ept, int rows_ept1, int col_threads, int km_ept,
           int km_ept1, int col_ept, int col_ept1)
{
    if (c.plan_block) (void)hipFree(c.plan_block);
    if (c.dir_block) (void)hipFree(c.dir_block);
    c.plan_block = c.dir_block = nullptr;
    c.tpw_up = tpw_up, c.tpw_dn = tpw_dn, c.xcd_pair = xcd_pair, c.rows_ept = rows_ept, c.rows_ept1 = rows_ept1,
    c.col_threads = col_threads, c.km_ept = km_ept, c.km_ept1 = km_ept1, c.col_ept = col_ept, c.col_ept1 = col_ept1;
    return build_plans(c);
}

int build_plans(Ctx& c)
{
    if (c.n_q > MAX_LAUNCH_LIMBS / 2 || c.n_q + c.n_p > 127)
        return set_error(-5, "too many primes for the launch maps");
    // a windowed context (levels of the 25-30 system) rescales rationally:
    // its rescaling plans merge ModDown into the rescaling to the window below
    auto planned = [&](int rs, int level) {
        return c.has_level(level) && (rs == 0 || (c.windowed ? c.rr_below[level] > 0 : level >= 2));
    };
    Blob b;
    for (int rs = 0; rs < 2; rs++) {
        c.ks_plan[rs].assign(c.n_q + 1, KsPlan{});
        for (int level = 1; level <= c.n_q; level++)
            if (planned(rs, level)) build_ks_plan(c, b, level, rs == 1, c.ks_plan[rs][level]);
    }
    c.rs_plan.assign(c.n_q + 1, RsPlan{});
    if (!c.windowed)
        for (int level = 2; level <= c.n_q; level++) build_rs_plan(c, b, level, c.rs_plan[level]);
    c.rr_plan.assign(c.n_q + 1, RrPlan{});
    for (int level = 1; level <= c.n_q && c.windowed; level++)
        if (c.has_level(level) && c.rr_below[level]) build_rr_plan(c, b, level, c.rr_plan[level]);
    if (hipMalloc(&c.plan_block, b.bytes.size()) != hipSuccess) return set_error(-4, "hipMalloc of launch plans failed");
    if (hipMemcpy(c.plan_block, b.bytes.data(), b.bytes.size(), hipMemcpyHostToDevice) != hipSuccess)
        return set_error(-4, "uploading launch plans failed");
    char* base = static_cast<char*>(c.plan_block);
    auto fix = [&](MapRef& m) { if (m.n || m.dev) rebase(m.dev, base); };
    for (int rs = 0; rs < 2; rs++)
        for (int level = 1; level <= c.n_q; level++) {
            if (!planned(rs, level)) continue;
            KsPlan& P = c.ks_plan[rs][level];
            fix(P.up_rows), fix(P.up_cols), fix(P.dn_cols), fix(P.dn_rows), fix(P.up_nrows);
            for (auto& r : P.up_bc) rebase(r.dev, base);
            for (auto& r : P.dn_bc) rebase(r.dev, base);
        }
    for (int level = 2; level <= c.n_q && !c.windowed; level++) {
        RsPlan& P = c.rs_plan[level];
        fix(P.rows), fix(P.cols), fix(P.ncols), fix(P.nrows);
    }
    for (int level = 1; level <= c.n_q && c.windowed; level++) {
        RrPlan& P = c.rr_plan[level];
        if (!P.rows.n) continue;
        fix(P.rows), fix(P.cols), fix(P.nrows);
        for (auto& r : P.bc) rebase(r.dev, base);
    }
    // per-level directories for batched launches: 6 pointer arrays per rescale flag
    const size_t per = (size_t)c.n_q + 1;
    std::vector<const void*> dir(2 * 6 * per, nullptr);
    for (int rs = 0; rs < 2; rs++)
        for (int level = 1; level <= c.n_q; level++) {
            if (!planned(rs, level)) continue;
            const KsPlan& P = c.ks_plan[rs][level];
            const void** d = dir.data() + (size_t)rs * 6 * per;
            const bool one = P.up_bc.size() == 1 && P.dn_bc.size() == 1;
            d[0 * per + level] = P.up_rows.dev;
            d[1 * per + level] = P.up_cols.dev;
            d[2 * per + level] = one ? (const void*)P.up_bc[0].dev : nullptr;
            d[3 * per + level] = P.dn_cols.dev;
            d[4 * per + level] = one ? (const void*)P.dn_bc[0].dev : nullptr;
            d[5 * per + level] = P.dn_rows.dev;
        }
    if (hipMalloc(&c.dir_block, dir.size() * sizeof(void*)) != hipSuccess)
        return set_error(-4, "hipMalloc of plan directory failed");
    if (hipMemcpy(c.dir_block, dir.data(), dir.size() * sizeof(void*), hipMemcpyHostToDevice) != hipSuccess)
        return set_error(-4, "uploading plan directory failed");
    for (int rs = 0; rs < 2; rs++) {
        const void* const* d = static_cast<const void* const*>(c.dir_block) + (size_t)rs * 6 * per;
        KsDir& D = c.ks_dir[rs];
        D.up_rows = reinterpret_cast<const LaunchMap* const*>(d + 0 * per);
        D.up_cols = reinterpret_cast<const LaunchMap* const*>(d + 1 * per);
        D.up_bc = reinterpret_cast<const BcMap* const*>(d + 2 * per);
        D.dn_cols = reinterpret_cast<const LaunchMap* const*>(d + 3 * per);
        D.dn_bc = reinterpret_cast<const BcMap* const*>(d + 4 * per);
        D.dn_rows = reinterpret_cast<const LaunchMap* const*>(d + 5 * per);
    }
    return 0;
}

}  // namespace ckks
