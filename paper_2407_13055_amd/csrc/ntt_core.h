// Negacyclic NTT / INTT building blocks for gfx950 (Sec. 2.2; Sec. 4.2
// "(I)NTT ... stages split into phases").
//
// Transform (bit-reversed evaluation order):
//     A[k] = sum_n a[n] * psi^((2*brev(k)+1)*n)  (mod q)
// computed by the merged Cooley-Tukey recursion: stage s (0 <= s < log N)
// pairs j and j + N/2^(s+1) inside block i = j >> (log N - s) with twiddle
// Psi[2^s + i] = psi^brev(2^s + i); the inverse runs Gentleman-Sande stages
// in reverse with inverse twiddles and folds N^-1 (and any constant that
// follows, Sec. 5.1 Seq.1/Seq.2) into its last stage.
//
// Decomposition of one limb of N = 2^LOG1 * 256 residues, viewed as a
// 2^LOG1 x 256 row-major matrix (index j = h*256 + l):
//   column pass: stages 0 .. LOG1-1 act on h for each column l;
//   row pass   : stages LOG1 .. log N - 1 act on l for each row h.
// Each pass is one kernel; 256 threads each hold 16 residues in VGPRs and
// run up to four radix-2 stages in registers ("round"), exchange once
// through LDS, and run the remaining stages.  One pass reads and writes the
// limb once; the 255 twiddles of the column pass are shared by every column
// (wave-uniform loads), the row pass reads each row's own 255 twiddles.
#pragma once
#include <type_traits>

#include "internal.h"
#include "modarith.h"

namespace ckks {

constexpr int ROW_LOG = 8;
constexpr int ROW = 1 << ROW_LOG;
constexpr int NTT_THREADS = 256;
constexpr int ROWS_PER_WG = NTT_THREADS / 16;  // row pass: 16 threads per row

// ---------------------------------------------------------------------------
// Butterflies with Shoup twiddles (w, floor(w 2^32/q)) and lazy ranges.
// Two classes of primes, chosen per work-group (uniform branch):
//   q < 2^30 ("wide"): forward stages keep values in [0, 4q), inverse
//     stages in [0, 2q): 3 multiplies + 5 or 6 adds per butterfly.
//   q >= 2^30 (31-bit): 4q overflows 32 bits, so forward values stay in
//     [0, 2q) and inverse values canonical: 3 multiplies + 7 adds.
// Pass boundaries: a forward column pass hands the row pass values in the
// forward range; a forward row pass and an inverse column pass end with a
// reduction to [0, q); an inverse row pass hands the column pass values in
// the inverse range.  Inputs read from memory are canonical.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool wide_prime(uint32_t q) { return q < (1u << 30); }

// in-register radix-2 stages over the low NS bits of the register index k
// (x[k], k < E; E = 16, or 4 in the wave-per-row passes).  tw(u, b) returns the Shoup twiddle of stage u for
// register block b = k >> (NS - u).
template <int NS, bool WIDE, class TW, int E>
__device__ __forceinline__ void ct_stages(uint32_t (&x)[E], uint32_t q, TW&& tw)
{
    const uint32_t q2 = 2 * q;
#pragma unroll
    for (int u = 0; u < NS; u++) {
        const int half = 1 << (NS - 1 - u), span = 2 * half;
#pragma unroll
        for (int b = 0; b < E / span; b++) {
            const uint2 w = tw(u, b);
#pragma unroll
            for (int m = 0; m < half; m++) {
                const int k = b * span + m;
                if constexpr (WIDE) {  // [0, 4q) -> [0, 4q)
                    // nt = -t (mod 2^32) for the Shoup product t in [0, 2q):
                    // a + t = a - nt, and a - t + 2q is one three-input add
                    const uint32_t a = red2(x[k], q2);
                    const uint32_t nt = mul_shoup_neg(x[k + half], w.x, w.y, q);
                    x[k] = a - nt;
                    x[k + half] = a + nt + q2;
                } else {               // [0, 2q) -> [0, 2q)
                    const uint32_t a = red2(x[k], q);
                    const uint32_t t = red2(mul_shoup(x[k + half], w.x, w.y, q), q);
                    x[k] = a + t;
                    x[k + half] = a - t + q;
                }
            }
        }
    }
}

// forward range -> [0, q)
template <bool WIDE, int E>
__device__ __forceinline__ void ct_canon(uint32_t (&x)[E], uint32_t q)
{
#pragma unroll
    for (int k = 0; k < E; k++) x[k] = red2(WIDE ? red2(x[k], 2 * q) : x[k], q);
}

// Gentleman-Sande inverse stages, u = NS-1 .. 0.  If FOLD, stage u == 0 also
// multiplies both outputs by a constant: c = (c, c_shoup, c w, (c w)_shoup)
// with w the stage-0 twiddle, and ends canonical.
template <int NS, bool WIDE, bool FOLD, class TW, int E>
__device__ __forceinline__ void gs_stages(uint32_t (&x)[E], uint32_t q, TW&& tw, uint4 c = uint4{0, 0, 0, 0})
{
    const uint32_t q2 = 2 * q;
#pragma unroll
    for (int u = NS - 1; u >= 0; u--) {
        const int half = 1 << (NS - 1 - u), span = 2 * half;
#pragma unroll
        for (int b = 0; b < E / span; b++) {
            const uint2 w = (FOLD && u == 0) ? make_uint2(c.z, c.w) : tw(u, b);
#pragma unroll
            for (int m = 0; m < half; m++) {
                const int k = b * span + m;
                const uint32_t a = x[k], y = x[k + half];
                if constexpr (WIDE) {  // [0, 2q) -> [0, 2q)
                    if (FOLD && u == 0) {
                        x[k] = red2(mul_shoup(a + y, c.x, c.y, q), q);
                        x[k + half] = red2(mul_shoup(a + q2 - y, w.x, w.y, q), q);
                    } else {
                        x[k] = red2(a + y, q2);
                        x[k + half] = mul_shoup(a + q2 - y, w.x, w.y, q);
                    }
                } else {               // [0, q) -> [0, q)
                    if (FOLD && u == 0) {
                        x[k] = red2(mul_shoup(a + y, c.x, c.y, q), q);
                    } else {
                        x[k] = red2(a + y, q);
                    }
                    x[k + half] = red2(mul_shoup(a + q - y, w.x, w.y, q), q);
                }
            }
        }
    }
}

// Calls f(tag) with tag = std::integral_constant<bool, q < 2^30>: q is
// uniform across the work-group, so this is one branch and each prime class
// gets its own straight-line code (read the class as
// decltype(tag)::value).
template <class F>
__device__ __forceinline__ void by_class(uint32_t q, F&& f)
{
    if (wide_prime(q))
        f(std::integral_constant<bool, true>{});
    else
        f(std::integral_constant<bool, false>{});
}

// ---------------------------------------------------------------------------
// LDS exchange layouts (one padding slot per 16 entries keeps both access
// patterns free of bank conflicts).
// ---------------------------------------------------------------------------
// column pass: element (row h, column c) of a 2^LOG1 x C tile
template <int C>
__device__ __forceinline__ int col_lds(int h, int c) { return (h + (h >> 4)) * C + c; }
// row pass: element (row rr, column l) of a 16 x 256 tile
__device__ __forceinline__ int row_lds(int rr, int l) { return rr * (ROW + ROW / 16) + l + (l >> 4); }

// Column tile of CT threads (256, or 512 for 128-byte rows at N = 2^16):
// 16 residues per thread, R threads per column, C columns.
template <int LOG1, int CT = NTT_THREADS>
struct ColGeom {
    static constexpr int S1 = 1 << LOG1;        // points per column transform
    static constexpr int R = S1 / 16;           // threads per column
    static constexpr int C = CT / R;            // columns per work-group
    static constexpr int NS2 = LOG1 - 4;        // stages in the second round
    static constexpr int LDS = (S1 + S1 / 16) * C;
    static constexpr int TILE = CT * 16;        // residues per tile (tile-thread layout)
    static_assert(C <= ROW, "column tile wider than a row");
};
constexpr int ROW_LDS_WORDS = ROWS_PER_WG * (ROW + ROW / 16);

// Launch geometry shared by all passes: blockIdx.y = limb of the launch,
// blockIdx.x = tile (column block or row block) inside the limb.
template <int LOG1, int CT = NTT_THREADS>
__host__ __device__ constexpr int col_tiles() { return ROW / ColGeom<LOG1, CT>::C; }

// Column tile of a column-pass work-group.  Work-groups go to the 8 XCDs
// round-robin in launch order (blockIdx.x fastest), so tile = blockIdx.x
// would put the two 64-byte halves of a 128-byte line (tiles 2m, 2m+1 when
// a tile is 16 columns) on different XCDs and fetch every line twice; pair
// them on one XCD instead.
template <int LOG1, int CT = NTT_THREADS>
__device__ __forceinline__ int col_tile(int pair)
{
    constexpr int T = col_tiles<LOG1, CT>();
    if constexpr (T == 16)
        return pair ? 2 * (blockIdx.x & 7) + (blockIdx.x >> 3) : (int)blockIdx.x;
    else if constexpr (T == 32)  // 8-column tiles: four per 128-byte line
        return pair ? 4 * (blockIdx.x & 7) + (blockIdx.x >> 3) : (int)blockIdx.x;
    else
        return blockIdx.x;
}
template <int LOG1>
__host__ __device__ constexpr int row_tiles() { return (1 << LOG1) / ROWS_PER_WG; }

// ---------------------------------------------------------------------------
// Pass kernels.  Ld::at(item) / St::at(item) return copies whose pointers
// are advanced to batch item `item` (identity for a single operation).
// Ld::load(M, limb, j, pc) / Ld::load16(M, limb, j0, pc, x)
// produce input residues (fused prologues); St::store(M, limb, j, v, pc) /
// St::store16 consume outputs (fused epilogues); St::final_const(M, limb) is
// the constant folded into the last inverse stage.  M.pid[limb] is the prime.
// ---------------------------------------------------------------------------
struct PrimeC {
    uint32_t q, qinv;
};

// Launch maps reach the kernels either by value (kernel argument; the
// stand-alone NTT call with caller-chosen primes) or as a pointer to a map
// precomputed in device memory at context creation (every internal launch:
// a 2 KB kernel argument costs more per launch than the kernel's own start).
struct MapByVal {
    LaunchMap m;
    __device__ const LaunchMap* get() const { return &m; }
};
struct MapByPtr {
    const LaunchMap* p;
    __device__ const LaunchMap* get() const { return p; }
};
// batched launch: item blockIdx.z uses the map of its own level; an item
// whose level lies outside [lo, hi], whose key index lies outside
// [0, n_keys) or whose input slot lies outside [0, n_src) gets no map and is
// skipped by every pass (n_src == 0: the launch reads one shared input and
// ignores the slot)
__device__ __forceinline__ bool item_ok(const BatchItem& it, int lo, int hi, int n_keys, int n_src)
{
    return it.level >= lo && it.level <= hi && it.key >= 0 && it.key < n_keys &&
           (n_src == 0 || (it.src >= 0 && it.src < n_src));
}
struct MapDir {
    const LaunchMap* const* dir;
    const BatchItem* items;
    int lo, hi, n_keys, n_src;
    __device__ const LaunchMap* get() const
    {
        const BatchItem it = items[blockIdx.z];
        return item_ok(it, lo, hi, n_keys, n_src) ? dir[it.level] : nullptr;
    }
};

struct NttTables {
    const uint2* tw;        // [n_primes][N] Shoup pairs of Psi (forward) or Psi^-1 (inverse)
    const uint32_t* twq;    // [n_primes][N] the same twiddles as floor(w 2^32 / q) alone
    const uint32_t* mods;   // [n_primes]
    const uint32_t* qinvs;  // [n_primes] q^-1 mod 2^32
    int log_n;
    int xcd_pair;           // column-tile order (col_tile)
};

// Row-pass twiddles of a work-group's ROWS_PER_WG rows, staged in LDS (one
// slot per thread) for kernels that run the same row pass several times
// (KeyMult: once per digit).  Row i, slot s: s < 15 is the first round
// (stage u = log2(s+1), block s+1-2^u: read at (1 << u) - 1 + b); s >= 16 is
// the second round (stage u = log2(s)-4, local index (rp << u) + b: read at
// (16 << u) + (rp << u) + b).  Ends with a barrier.
//
// The entries are generated, not loaded (on-the-fly twiddles, Sec. 4.2): the
// table holds psi^brev(i), and the index of a row-pass twiddle splits into
// disjoint bit fields, high = 2^(LOG1+lg) + (h << lg) and low = loc < 2^lg,
// so psi^brev(i) = psi^brev(high) * psi^brev(low): two table entries shared
// by many slots, one Shoup product, and the Shoup companion
// floor(w 2^32 / q) from a double-precision estimate corrected exactly by
// one step.  The work-group reads 2 KB of table instead of 32 KB.
constexpr int ROW_TW_SLOTS = 256;
template <int LOG1>
__device__ __forceinline__ void stage_row_twiddles(uint2* tws, const uint2* tw, int h0, uint32_t q)
{
    static_assert(NTT_THREADS == ROW_TW_SLOTS, "one slot per thread");
    const int sl = threadIdx.x;
    if (sl != 15) {
        const int lg = 31 - __clz(sl < 15 ? sl + 1 : sl);
        const int loc = sl < 15 ? sl + 1 - (1 << lg) : sl - (1 << lg);
        const uint2 lo = tw[loc];
        const double rq = 4294967296.0 / (double)q;
#pragma unroll 4
        for (int i = 0; i < ROWS_PER_WG; i++) {
            const uint32_t hi = tw[(1 << (LOG1 + lg)) + ((h0 + i) << lg)].x;
            const uint32_t w = red2(mul_shoup(hi, lo.x, lo.y, q), q);
            uint32_t ws = (uint32_t)((double)w * rq);  // floor(w 2^32 / q) or one off
            const int64_t r = (int64_t)((uint64_t)w << 32) - (int64_t)((uint64_t)ws * q);
            ws = r < 0 ? ws - 1 : (r >= (int64_t)q ? ws + 1 : ws);
            tws[i * ROW_TW_SLOTS + sl] = make_uint2(w, ws);
        }
    }
    __syncthreads();
}
__device__ __forceinline__ uint2 row_tw1(const uint2* tws, int rr, int u, int b) { return tws[rr * ROW_TW_SLOTS + (1 << u) - 1 + b]; }
__device__ __forceinline__ uint2 row_tw2(const uint2* tws, int rr, int rp, int u, int b)
{
    return tws[rr * ROW_TW_SLOTS + (16 << u) + (rp << u) + b];
}

// forward, column pass (stages 0 .. LOG1-1)
template <int LOG1, class MS, class Ld, class St, int CT = NTT_THREADS>
__global__ void __launch_bounds__(CT) k_fwd_cols(NttTables T, MS ms, Ld ld0, St st0)
{
    // grid.z = batch item; grid.y is sized for the largest map of a batch
    const LaunchMap* Mp = ms.get();
    if (!Mp || (int)blockIdx.y >= Mp->count) return;
    const LaunchMap& M = *Mp;
    const Ld ld = ld0.at(blockIdx.z);
    const St st = st0.at(blockIdx.z);
    using G = ColGeom<LOG1, CT>;
    __shared__ uint32_t lds[G::LDS];
    const int limb = blockIdx.y, pid = M.pid[limb];
    const uint32_t q = T.mods[pid];
    const PrimeC pc{q, T.qinvs[pid]};
    const uint2* tw = T.tw + ((size_t)pid << T.log_n);
    const int c = threadIdx.x % G::C, r = threadIdx.x / G::C;
    const int col = col_tile<LOG1, CT>(T.xcd_pair) * G::C + c;
    uint32_t x[16];
    if constexpr (Ld::kTileThread) {
        ld.load16(M, limb, col_tile<LOG1, CT>(T.xcd_pair) * G::TILE + threadIdx.x * 16, pc, x);
    } else {
#pragma unroll
        for (int k = 0; k < 16; k++) x[k] = ld.load(M, limb, (r + G::R * k) * ROW + col, pc);
    }
    by_class(q, [&](auto tag) {
        constexpr bool W = decltype(tag)::value;
        ct_stages<4, W>(x, q, [&](int u, int b) { return tw[(1 << u) + b]; });
        if constexpr (G::NS2 > 0) {
#pragma unroll
            for (int k = 0; k < 16; k++) lds[col_lds<G::C>(r + G::R * k, c)] = x[k];
            __syncthreads();
#pragma unroll
            for (int k = 0; k < 16; k++) x[k] = lds[col_lds<G::C>(16 * r + k, c)];
            ct_stages<G::NS2, W>(x, q, [&](int u, int b) {
                return tw[(1 << (4 + u)) + (r << (4 - G::NS2 + u)) + b];
            });
#pragma unroll
            for (int k = 0; k < 16; k++) st.store(M, limb, (16 * r + k) * ROW + col, x[k], pc);
        } else {
#pragma unroll
            for (int k = 0; k < 16; k++) st.store(M, limb, (r + G::R * k) * ROW + col, x[k], pc);
        }
    });
}

// forward, row pass (stages LOG1 .. LOG1+7); ends canonical
template <int LOG1, class MS, class Ld, class St>
__global__ void __launch_bounds__(NTT_THREADS) k_fwd_rows(NttTables T, MS ms, Ld ld0, St st0)
{
    // grid.z = batch item; grid.y is sized for the largest map of a batch
    const LaunchMap* Mp = ms.get();
    if (!Mp || (int)blockIdx.y >= Mp->count) return;
    const LaunchMap& M = *Mp;
    const Ld ld = ld0.at(blockIdx.z);
    const St st = st0.at(blockIdx.z);
    __shared__ uint32_t lds[ROW_LDS_WORDS];
    const int limb = blockIdx.y, pid = M.pid[limb];
    const uint32_t q = T.mods[pid];
    const PrimeC pc{q, T.qinvs[pid]};
    const uint2* tw = T.tw + ((size_t)pid << T.log_n);
    const int rp = threadIdx.x % 16, rr = threadIdx.x / 16;
    const int h = blockIdx.x * ROWS_PER_WG + rr;  // 2^LOG1 rows, LOG1 >= 4: exact grid
    uint32_t x[16];
#pragma unroll
    for (int k = 0; k < 16; k++) x[k] = ld.load(M, limb, h * ROW + rp + 16 * k, pc);
    by_class(q, [&](auto tag) {
        constexpr bool W = decltype(tag)::value;
        ct_stages<4, W>(x, q, [&](int u, int b) { return tw[(1 << (LOG1 + u)) + (h << u) + b]; });
#pragma unroll
        for (int k = 0; k < 16; k++) lds[row_lds(rr, rp + 16 * k)] = x[k];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 16; k++) x[k] = lds[row_lds(rr, 16 * rp + k)];
        ct_stages<4, W>(x, q, [&](int u, int b) {
            return tw[(1 << (LOG1 + 4 + u)) + (h << (4 + u)) + (rp << u) + b];
        });
        ct_canon<W>(x, q);
    });
    st.store16(M, limb, h * ROW + 16 * rp, x, pc);
}

// inverse, row pass (stages LOG1+7 .. LOG1)
template <int LOG1, class MS, class Ld, class St>
__global__ void __launch_bounds__(NTT_THREADS) k_inv_rows(NttTables T, MS ms, Ld ld0, St st0)
{
    // grid.z = batch item; grid.y is sized for the largest map of a batch
    const LaunchMap* Mp = ms.get();
    if (!Mp || (int)blockIdx.y >= Mp->count) return;
    const LaunchMap& M = *Mp;
    const Ld ld = ld0.at(blockIdx.z);
    const St st = st0.at(blockIdx.z);
    __shared__ uint32_t lds[ROW_LDS_WORDS];
    const int limb = blockIdx.y, pid = M.pid[limb];
    const uint32_t q = T.mods[pid];
    const PrimeC pc{q, T.qinvs[pid]};
    const uint2* tw = T.tw + ((size_t)pid << T.log_n);
    const int rp = threadIdx.x % 16, rr = threadIdx.x / 16;
    const int h = blockIdx.x * ROWS_PER_WG + rr;
    uint32_t x[16];
    ld.load16(M, limb, h * ROW + 16 * rp, pc, x);
    by_class(q, [&](auto tag) {
        constexpr bool W = decltype(tag)::value;
        gs_stages<4, W, false>(x, q, [&](int u, int b) {
            return tw[(1 << (LOG1 + 4 + u)) + (h << (4 + u)) + (rp << u) + b];
        });
#pragma unroll
        for (int k = 0; k < 16; k++) lds[row_lds(rr, 16 * rp + k)] = x[k];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 16; k++) x[k] = lds[row_lds(rr, rp + 16 * k)];
        gs_stages<4, W, false>(x, q, [&](int u, int b) { return tw[(1 << (LOG1 + u)) + (h << u) + b]; });
    });
#pragma unroll
    for (int k = 0; k < 16; k++) st.store(M, limb, h * ROW + rp + 16 * k, x[k], pc);
}

// ---------------------------------------------------------------------------
// Row passes with one wave per row (4 residues per thread, 4 rows per
// work-group): four radix-4 rounds with three exchanges, through the wave's
// own LDS row or in registers.  Four times the waves of the 16-residue
// passes: more memory latency hidden per SIMD when a launch has few limbs.
// Round j of the forward pass holds the 4 points
// l = blk*2^(sh+2) + pp + k*2^sh (sh = 6 - 2j, blk = t >> sh); the inverse
// pass walks the same units in the opposite order (sh = 2j).  A round stores
// its results where it read its inputs, and each point is read by one lane
// per round, so one buffer serves every round.  Only the wave itself touches
// its row, and a CU performs one wave's LDS operations in issue order, so
// the exchanges need no work-group barrier: wave_lds_sync only keeps the
// compiler from moving LDS accesses across the exchange.
// ---------------------------------------------------------------------------
constexpr int ROWS4 = NTT_THREADS / 64;   // rows (waves) per work-group
// the wave's index in its work-group, as a scalar (the same in every lane)
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }
constexpr int ROW4_PITCH = ROW + ROW / 16;
__device__ __forceinline__ int row4_lds(int w, int l) { return w * ROW4_PITCH + l + (l >> 4); }
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
template <int LOG1>
__host__ __device__ constexpr int row4_tiles() { return (1 << LOG1) / ROWS4; }

// 4 x 4 transpose across the lanes of each quad, in registers: lane a's
// register b becomes lane b's register a.  Two exchange stages with the
// partner lane (DPP quad permutes): first the entries whose lane and register
// indices differ in bit 0 (partner lane a^1, register b^1), then in bit 1.
__device__ __forceinline__ void quad_transpose(uint32_t (&x)[4], int lane)
{
    constexpr int SWAP1 = 1 | (0 << 2) | (3 << 4) | (2 << 6);  // quad_perm [1, 0, 3, 2]
    constexpr int SWAP2 = 2 | (3 << 2) | (0 << 4) | (1 << 6);  // quad_perm [2, 3, 0, 1]
    uint32_t y[4];
#pragma unroll
    for (int b = 0; b < 4; b++) y[b] = (uint32_t)__builtin_amdgcn_mov_dpp((int)x[b ^ 1], SWAP1, 0xF, 0xF, true);
#pragma unroll
    for (int b = 0; b < 4; b++) x[b] = ((b ^ lane) & 1) ? y[b] : x[b];
#pragma unroll
    for (int b = 0; b < 4; b++) y[b] = (uint32_t)__builtin_amdgcn_mov_dpp((int)x[b ^ 2], SWAP2, 0xF, 0xF, true);
#pragma unroll
    for (int b = 0; b < 4; b++) x[b] = ((b ^ lane) & 2) ? y[b] : x[b];
}

// Forward row pass of the row a wave holds: x[k] = row[t + 64 k] on entry,
// row[4 t + k] on exit (canonical); tw[j][i]: round j's twiddles (stage 0,
// then the two of stage 1).  The exchanges after rounds 0 and 1 go through
// the wave's LDS row; between rounds 2 and 3 the 16 points of a quad of
// lanes (lane a of quad m holds 16m + a + 4k, and needs 16m + 4a + k) change
// places with a quad transpose in registers.  SYNC0: order the pass after a
// previous pass over the same LDS row.
template <bool W, bool SYNC0 = true>
__device__ __forceinline__ void row4_fwd(uint32_t (&x)[4], uint32_t q, uint32_t* lds, int w, int t,
                                         const uint2 (&tw)[4][3])
{
    if (SYNC0) wave_lds_sync();
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const int sh = 6 - 2 * j, pp = t & ((1 << sh) - 1);
        const int l0 = ((t >> sh) << (sh + 2)) + pp;
        if (j == 3) {
            quad_transpose(x, t);
        } else if (j) {
            wave_lds_sync();
#pragma unroll
            for (int k = 0; k < 4; k++) x[k] = lds[row4_lds(w, l0 + (k << sh))];
        }
        ct_stages<2, W>(x, q, [&](int u, int b) { return tw[j][u ? 1 + b : 0]; });
        if (j < 2) {
#pragma unroll
            for (int k = 0; k < 4; k++) lds[row4_lds(w, l0 + (k << sh))] = x[k];
        }
    }
    ct_canon<W>(x, q);
}

// Inverse row pass: x[k] = row[4 t + k] on entry, row[t + 64 k] on exit
// (inverse range); tw[j][i] as in row4_fwd for round j of the inverse.  The
// exchange between rounds 0 and 1 is the quad transpose (the forward pass's
// last one, undone).
template <bool W, bool SYNC0 = true>
__device__ __forceinline__ void row4_inv(uint32_t (&x)[4], uint32_t q, uint32_t* lds, int w, int t,
                                         const uint2 (&tw)[4][3])
{
    if (SYNC0) wave_lds_sync();
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const int sh = 2 * j, pp = t & ((1 << sh) - 1);
        const int l0 = ((t >> sh) << (sh + 2)) + pp;
        if (j == 1) {
            quad_transpose(x, t);
        } else if (j) {
            wave_lds_sync();
#pragma unroll
            for (int k = 0; k < 4; k++) x[k] = lds[row4_lds(w, l0 + (k << sh))];
        }
        gs_stages<2, W, false>(x, q, [&](int u, int b) { return tw[j][u ? 1 + b : 0]; });
        if (j >= 1 && j < 3) {
#pragma unroll
            for (int k = 0; k < 4; k++) lds[row4_lds(w, l0 + (k << sh))] = x[k];
        }
    }
}

// The Shoup pair (w, ws) of a twiddle stored as ws = floor(w 2^32 / q)
// alone (0 <= w < q < 2^32): w 2^32 lies in [ws q, ws q + q), so w lies in
// [ws q / 2^32, (ws q + q) / 2^32), an interval shorter than 1; the one
// integer there is ceil(ws q / 2^32).
__device__ __forceinline__ uint2 shoup_from_quot(uint32_t ws, uint32_t q)
{
    const uint32_t lo = ws * q, hi = __umulhi(ws, q);
    return make_uint2(hi + (lo != 0u ? 1u : 0u), ws);
}

// the twiddles thread t uses in row h (forward: round j covers stages
// LOG1 + 2j, LOG1 + 2j + 1; inverse: the same stages in reverse order).
// h is the same in every lane of a wave, so each entry's address is a
// wave-uniform base plus a 32-bit lane offset (scalar-base loads).
template <int LOG1, bool INV>
__device__ __forceinline__ void row4_twiddles(const uint2* tw, int h, int t, uint2 (&out)[4][3])
{
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const int g = INV ? 6 - 2 * j : 2 * j;         // stage offset of the round's first stage
        const uint32_t blk = (uint32_t)t >> (INV ? 2 * j : 6 - 2 * j);
        const uint2* s0 = tw + ((1u << (LOG1 + g)) + ((uint32_t)h << g));
        const uint2* s1 = tw + ((1u << (LOG1 + g + 1)) + ((uint32_t)h << (g + 1)));
        out[j][0] = s0[blk];
#pragma unroll
        for (int b = 0; b < 2; b++) out[j][1 + b] = s1[(blk << 1) + (uint32_t)b];
    }
}

// the same twiddles read from the quotient-only table twq of prime q (4
// bytes per entry; two multiplies per twiddle recover w): for a kernel that
// reuses them (KeyMult, once per digit), where the halved table traffic pays
template <int LOG1, bool INV>
__device__ __forceinline__ void row4_twiddles_q(const uint32_t* twq, uint32_t q, int h, int t, uint2 (&out)[4][3])
{
    uint32_t ws[4][3];
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const int g = INV ? 6 - 2 * j : 2 * j;         // stage offset of the round's first stage
        const uint32_t blk = (uint32_t)t >> (INV ? 2 * j : 6 - 2 * j);
        const uint32_t* s0 = twq + ((1u << (LOG1 + g)) + ((uint32_t)h << g));
        const uint32_t* s1 = twq + ((1u << (LOG1 + g + 1)) + ((uint32_t)h << (g + 1)));
        ws[j][0] = s0[blk];
#pragma unroll
        for (int b = 0; b < 2; b++) ws[j][1 + b] = s1[(blk << 1) + (uint32_t)b];
    }
#pragma unroll
    for (int j = 0; j < 4; j++)
#pragma unroll
        for (int i = 0; i < 3; i++) out[j][i] = shoup_from_quot(ws[j][i], q);
}

// Launch-map entries of a work-group's limb (scalar loads issued together;
// the entries of limbs at or above count are in bounds and unused).
struct LimbInfo {
    int count, pid;
    uint32_t q, qinv;
};
__device__ __forceinline__ LimbInfo limb_info(const NttTables& T, const LaunchMap& M, int limb)
{
    LimbInfo r;
    r.count = M.count;
    r.pid = M.pid[limb];
    r.q = T.mods[r.pid];
    r.qinv = T.qinvs[r.pid];
    return r;
}

// Row passes with one wave per row: every operand (the row, the twelve
// twiddles of the four rounds, and what the epilogue reads) is requested
// before the first wait, so a work-group pays about one memory latency.
template <int LOG1, class MS, class Ld, class St>
__global__ void __launch_bounds__(NTT_THREADS) k_fwd_rows4(NttTables T, MS ms, Ld ld0, St st0)
{
    const LaunchMap* Mp = ms.get();
    if (!Mp) return;
    const LaunchMap& M = *Mp;
    const int limb = blockIdx.y;
    const LimbInfo I = limb_info(T, M, limb);
    if (limb >= I.count) return;
    const Ld ld = ld0.at(blockIdx.z);
    const St st = st0.at(blockIdx.z);
    __shared__ uint32_t lds[ROWS4 * ROW4_PITCH];
    const PrimeC pc{I.q, I.qinv};
    const int t = threadIdx.x & 63, w = wave_id();
    const int h = blockIdx.x * ROWS4 + w;  // exact grid
    uint32_t x[4];
#pragma unroll
    for (int k = 0; k < 4; k++) x[k] = ld.load(M, limb, h * ROW + t + 64 * k, pc);
    uint2 tw[4][3];
    row4_twiddles<LOG1, false>(T.tw + ((size_t)I.pid << T.log_n), h, t, tw);
    const auto pre = st.template prefetch<4>(M, limb, h * ROW + 4 * t);
    by_class(I.q, [&](auto tag) { row4_fwd<decltype(tag)::value, false>(x, I.q, lds, w, t, tw); });
    st.template storev<4>(M, limb, h * ROW + 4 * t, x, pc, pre);
}

template <int LOG1, class MS, class Ld, class St>
__global__ void __launch_bounds__(NTT_THREADS) k_inv_rows4(NttTables T, MS ms, Ld ld0, St st0)
{
    const LaunchMap* Mp = ms.get();
    if (!Mp) return;
    const LaunchMap& M = *Mp;
    const int limb = blockIdx.y;
    const LimbInfo I = limb_info(T, M, limb);
    if (limb >= I.count) return;
    const Ld ld = ld0.at(blockIdx.z);
    const St st = st0.at(blockIdx.z);
    __shared__ uint32_t lds[ROWS4 * ROW4_PITCH];
    const PrimeC pc{I.q, I.qinv};
    const int t = threadIdx.x & 63, w = wave_id();
    const int h = blockIdx.x * ROWS4 + w;
    uint32_t x[4];
    ld.template loadv<4>(M, limb, h * ROW + 4 * t, pc, x);
    uint2 tw[4][3];
    row4_twiddles<LOG1, true>(T.tw + ((size_t)I.pid << T.log_n), h, t, tw);
    by_class(I.q, [&](auto tag) { row4_inv<decltype(tag)::value, false>(x, I.q, lds, w, t, tw); });
#pragma unroll
    for (int k = 0; k < 4; k++) st.store(M, limb, h * ROW + t + 64 * k, x[k], pc);
}

// ---------------------------------------------------------------------------
// Column passes with 4 residues per thread.  256 threads hold a tile of
// C = 1024 / 2^LOG1 columns; thread (c = tid % C, t = tid / C) holds four
// points of column c.  Radix-4 rounds (plus one radix-2 round when LOG1 is
// odd) exchange through LDS, one barrier per exchange: four times the waves
// of the 16-residue passes.  In a radix-4 round with shift sh the thread's
// points are base + k 2^sh, base = ((t >> sh) << (sh + 2)) | (t mod 2^sh);
// the radix-2 round holds 4t + k.  The forward pass enters with points
// t + k TC (TC = 2^LOG1 / 4) and leaves with 4t + k; the inverse pass the
// other way round.  Tile-thread layout of lifted residues (the inverse pass
// writes it, the BConv pass reads it): thread tid of tile T keeps its four
// residues at T 1024 + 4 tid.
// ---------------------------------------------------------------------------
template <int LOG1>
struct Col4 {
    static constexpr int S1 = 1 << LOG1;           // points per column
    static constexpr int TC = S1 / 4;              // threads per column
    static constexpr int C = NTT_THREADS / TC;     // columns per work-group
    static constexpr int TILES = ROW / C;          // tiles per limb
    static constexpr int TILE = NTT_THREADS * 4;   // residues per tile
    static constexpr int NR4 = LOG1 / 2;           // radix-4 rounds
    static constexpr bool ODD = (LOG1 & 1) != 0;   // plus one radix-2 round
    static constexpr int NR = NR4 + (ODD ? 1 : 0);
    // LDS word of point p, column c: an additive padding, so the four
    // points of a round sit at fixed offsets from the first, chosen by
    // simulating every round's accesses (at most 2-way bank conflicts)
    static constexpr int PS = LOG1 == 8 ? 4 : 2;
    static constexpr int PA = LOG1 == 8 ? 12 : (LOG1 == 4 ? 0 : C);
    static constexpr int WORDS = S1 * C + PA * (S1 >> PS);  // one buffer
    __device__ static int lds(int p, int c) { return p * C + c + PA * (p >> PS); }
    // shift of forward round j (-1: the radix-2 round) and of inverse round j
    __host__ __device__ static constexpr int fsh(int j) { return j < NR4 ? LOG1 - 2 - 2 * j : -1; }
    __host__ __device__ static constexpr int ish(int j) { return ODD ? (j == 0 ? -1 : 1 + 2 * (j - 1)) : 2 * j; }
    static_assert(C >= 1 && C * TC == NTT_THREADS, "column tile");
};
__device__ __forceinline__ int col4_base(int t, int sh) { return sh < 0 ? 4 * t : (((t >> sh) << (sh + 2)) | (t & ((1 << sh) - 1))); }
__device__ __forceinline__ int col4_step(int sh) { return sh < 0 ? 1 : 1 << sh; }

// Column tile of a 4-residue column work-group: as col_tile, the tiles that
// share a 128-byte line run on one XCD.
template <int LOG1>
__device__ __forceinline__ int col4_tile(int pair)
{
    constexpr int T = Col4<LOG1>::TILES;
    if constexpr (T >= 16)
        return pair ? (T / 8) * (blockIdx.x & 7) + (blockIdx.x >> 3) : (int)blockIdx.x;
    else
        return blockIdx.x;
}

// A column pass uses the first 2^LOG1 - 1 twiddles of its prime's table
// (Psi[1 .. 2^LOG1 - 1], shared by every column): a work-group stages them
// in LDS once (one load per thread, 2 KB at N = 2^16) and every round reads
// them there.  Entry e of the staged copy is table entry e.  Ends with a
// barrier.
template <int LOG1, int NT>
__device__ __forceinline__ void col4_stage_twiddles(uint2* twl, const uint2* const (&tw)[NT])
{
#pragma unroll
    for (int i = 0; i < NT; i++)
        for (int e = threadIdx.x; e < (1 << LOG1); e += NTT_THREADS) twl[i * (1 << LOG1) + e] = tw[i][e];
    __syncthreads();
}
// twiddle of stage u of round j (sh: the round's shift) for pair block b
template <int LOG1>
__device__ __forceinline__ uint2 col4_tw(const uint2* twl, int t, int sh, int u, int b)
{
    if (sh < 0) return twl[(1 << (LOG1 - 1)) + 2 * t + b];  // radix-2 round: stage LOG1-1
    const int s0 = LOG1 - 2 - sh, blk = t >> sh;             // radix-4 round: stages s0, s0 + 1
    return twl[(1 << (s0 + u)) + (blk << u) + b];
}

// Forward column pass of NT targets held by the work-group: x[i] enters with
// points t + k TC of column c, leaves with 4t + k (canonical); lds holds
// one buffer of Col4::WORDS words per target (a round stores its results
// where it read its inputs, so one barrier per exchange suffices), twl the
// staged twiddles of each target
// (2^LOG1 entries apart).
template <int LOG1, int NT>
__device__ __forceinline__ void col4_fwd(uint32_t (&x)[NT][4], const uint32_t (&q)[NT], uint32_t* lds,
                                         const uint2* twl, int c, int t)
{
    using G = Col4<LOG1>;
#pragma unroll
    for (int j = 0; j < G::NR; j++) {
        const int sh = G::fsh(j), base = col4_base(t, sh), step = col4_step(sh);
        if (j) {
            __syncthreads();
#pragma unroll
            for (int i = 0; i < NT; i++)
#pragma unroll
                for (int k = 0; k < 4; k++) x[i][k] = lds[i * G::WORDS + G::lds(base + k * step, c)];
        }
#pragma unroll
        for (int i = 0; i < NT; i++) {
            const uint2* tl = twl + i * (1 << LOG1);
            by_class(q[i], [&](auto tag) {
                constexpr bool W = decltype(tag)::value;
                if (sh < 0)
                    ct_stages<1, W>(x[i], q[i], [&](int, int b) { return col4_tw<LOG1>(tl, t, sh, 0, b); });
                else
                    ct_stages<2, W>(x[i], q[i], [&](int u, int b) { return col4_tw<LOG1>(tl, t, sh, u, b); });
                if (j == G::NR - 1) ct_canon<W>(x[i], q[i]);
            });
        }
        if (j < G::NR - 1) {
#pragma unroll
            for (int i = 0; i < NT; i++)
#pragma unroll
                for (int k = 0; k < 4; k++) lds[i * G::WORDS + G::lds(base + k * step, c)] = x[i][k];
        }
    }
}

// Inverse column pass of one limb: x enters with points 4t + k, leaves with
// t + k TC, canonical, the last stage folding the constant cst (as
// gs_stages with FOLD).  lds: one buffer of Col4::WORDS words; twl: the
// staged inverse twiddles.
template <int LOG1, bool W>
__device__ __forceinline__ void col4_inv(uint32_t (&x)[4], uint32_t q, uint32_t* lds, const uint2* twl, int c, int t,
                                         uint4 cst)
{
    using G = Col4<LOG1>;
#pragma unroll
    for (int j = 0; j < G::NR; j++) {
        const int sh = G::ish(j), base = col4_base(t, sh), step = col4_step(sh);
        if (j) {
            __syncthreads();
#pragma unroll
            for (int k = 0; k < 4; k++) x[k] = lds[G::lds(base + k * step, c)];
        }
        const bool last = j == G::NR - 1;
        auto tw = [&](int u, int b) { return col4_tw<LOG1>(twl, t, sh, u, b); };
        if (sh < 0) {
            gs_stages<1, W, false>(x, q, [&](int, int b) { return tw(0, b); });
        } else if (last) {
            gs_stages<2, W, true>(x, q, tw, cst);
        } else {
            gs_stages<2, W, false>(x, q, tw);
        }
        if (!last) {
#pragma unroll
            for (int k = 0; k < 4; k++) lds[G::lds(base + k * step, c)] = x[k];
        }
    }
}

// inverse column pass, 4 residues per thread: reads the row-pass output,
// ends canonical with the constant folded, stores through St (tile-thread
// layout when St::kTileThread)
template <int LOG1, class MS, class Ld, class St>
__global__ void __launch_bounds__(NTT_THREADS) k_inv_cols4(NttTables T, MS ms, Ld ld0, St st0)
{
    using G = Col4<LOG1>;
    const LaunchMap* Mp = ms.get();
    if (!Mp) return;
    const LaunchMap& M = *Mp;
    const int limb = blockIdx.y;
    const LimbInfo I = limb_info(T, M, limb);
    if (limb >= I.count) return;
    const Ld ld = ld0.at(blockIdx.z);
    const St st = st0.at(blockIdx.z);
    __shared__ uint32_t lds[G::WORDS];
    __shared__ uint2 twl[1 << LOG1];
    const PrimeC pc{I.q, I.qinv};
    const int c = threadIdx.x % G::C, t = threadIdx.x / G::C;
    const int tile = col4_tile<LOG1>(T.xcd_pair), col = tile * G::C + c;
    uint32_t x[4];
#pragma unroll
    for (int k = 0; k < 4; k++) x[k] = ld.load(M, limb, (4 * t + k) * ROW + col, pc);
    const uint4 cst = st.final_const(M, limb);
    const uint2* const tws[1] = {T.tw + ((size_t)I.pid << T.log_n)};
    col4_stage_twiddles<LOG1, 1>(twl, tws);
    by_class(I.q, [&](auto tag) { col4_inv<LOG1, decltype(tag)::value>(x, I.q, lds, twl, c, t, cst); });
    if constexpr (St::kTileThread) {
        st.template storev<4>(M, limb, tile * G::TILE + threadIdx.x * 4, x, pc);
    } else {
#pragma unroll
        for (int k = 0; k < 4; k++) st.store(M, limb, (t + k * G::TC) * ROW + col, x[k], pc);
    }
}

// inverse, column pass (stages LOG1-1 .. 0); the last stage multiplies by
// st.final_const(M, limb) (N^-1 times whatever constant follows) and ends
// canonical.
template <int LOG1, class MS, class Ld, class St, int CT = NTT_THREADS>
__global__ void __launch_bounds__(CT) k_inv_cols(NttTables T, MS ms, Ld ld0, St st0)
{
    // grid.z = batch item; grid.y is sized for the largest map of a batch
    const LaunchMap* Mp = ms.get();
    if (!Mp || (int)blockIdx.y >= Mp->count) return;
    const LaunchMap& M = *Mp;
    const Ld ld = ld0.at(blockIdx.z);
    const St st = st0.at(blockIdx.z);
    using G = ColGeom<LOG1, CT>;
    __shared__ uint32_t lds[G::LDS];
    const int limb = blockIdx.y, pid = M.pid[limb];
    const uint32_t q = T.mods[pid];
    const PrimeC pc{q, T.qinvs[pid]};
    const uint2* tw = T.tw + ((size_t)pid << T.log_n);
    const int c = threadIdx.x % G::C, r = threadIdx.x / G::C;
    const int col = col_tile<LOG1, CT>(T.xcd_pair) * G::C + c;
    const uint4 cst = st.final_const(M, limb);
    uint32_t x[16];
    if constexpr (G::NS2 > 0) {
#pragma unroll
        for (int k = 0; k < 16; k++) x[k] = ld.load(M, limb, (16 * r + k) * ROW + col, pc);
    } else {
#pragma unroll
        for (int k = 0; k < 16; k++) x[k] = ld.load(M, limb, (r + G::R * k) * ROW + col, pc);
    }
    by_class(q, [&](auto tag) {
        constexpr bool W = decltype(tag)::value;
        if constexpr (G::NS2 > 0) {
            gs_stages<G::NS2, W, false>(x, q, [&](int u, int b) {
                return tw[(1 << (4 + u)) + (r << (4 - G::NS2 + u)) + b];
            });
#pragma unroll
            for (int k = 0; k < 16; k++) lds[col_lds<G::C>(16 * r + k, c)] = x[k];
            __syncthreads();
#pragma unroll
            for (int k = 0; k < 16; k++) x[k] = lds[col_lds<G::C>(r + G::R * k, c)];
        }
        gs_stages<4, W, true>(x, q, [&](int u, int b) { return tw[(1 << u) + b]; }, cst);
    });
    if constexpr (St::kTileThread) {
        // internal layout shared with the next column pass: thread tid of
        // tile t keeps its 16 residues at t*4096 + tid*16 (one 64-byte run)
        st.store16(M, limb, col_tile<LOG1, CT>(T.xcd_pair) * G::TILE + threadIdx.x * 16, x, pc);
    } else {
#pragma unroll
        for (int k = 0; k < 16; k++) st.store(M, limb, (r + G::R * k) * ROW + col, x[k], pc);
    }
}

}  // namespace ckks
