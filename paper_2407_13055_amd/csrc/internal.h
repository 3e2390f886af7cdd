// Library-internal declarations: the context (device tables built once per
// parameter set) and the launchers that the C-ABI entry points sequence.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <stdint.h>

#include <string>
#include <vector>

namespace ckks {

constexpr int MAX_PRIMES = 64;  // q's + p's
constexpr int MAX_LAUNCH_LIMBS = 128;

// Per-launch limb map (passed by value as a kernel argument, at most 4 KB).
// Launch limb l reads input limb in_off[l] and writes output limb
// out_off[l] (offsets in units of N residues from the functor's base
// pointer, output base chosen by grp[l]), has prime id pid[l], uses row
// cidx[l] of a constant table and matrix entries from mat_off[l];
// sub_off[l] addresses a second operand.  Every field is 32 bits wide so
// that a work-group reads its limb's entries with scalar loads (sub-word
// fields would take vector loads, one dependent memory round trip each).
struct LaunchMap {
    int32_t count;  // launch limbs in use (a batched launch sizes its grid for the largest level)
    int32_t in_off[MAX_LAUNCH_LIMBS];
    int32_t out_off[MAX_LAUNCH_LIMBS];
    int32_t sub_off[MAX_LAUNCH_LIMBS];
    int32_t mat_off[MAX_LAUNCH_LIMBS];
    int32_t cidx[MAX_LAUNCH_LIMBS];
    int32_t pid[MAX_LAUNCH_LIMBS];
    int32_t grp[MAX_LAUNCH_LIMBS];
};
static_assert(sizeof(LaunchMap) <= 4096, "a launch map must fit a kernel argument");

// Base-conversion launch map: groups of target primes sharing input rows
// (32-bit fields, as LaunchMap).
constexpr int MAX_BC_GROUPS = 128;
// zero entries after the last row of every BConv matrix: a kernel may read a
// whole chunk of this many constants past a group's last input
constexpr int BCONV_MAT_PAD = 8;
struct BcMap {
    int32_t groups;                     // groups in use
    int32_t in_off[MAX_BC_GROUPS];      // first input row of the group (units of N) in y
    int32_t first[MAX_BC_GROUPS];       // first target of the group
    int32_t n_in[MAX_BC_GROUPS];        // input rows
    int32_t n_tg[MAX_BC_GROUPS];        // targets in the group (<= targets per work-group)
    int32_t mat_off[MAX_LAUNCH_LIMBS];  // per target: constants at mat[mat_off + s]
    int32_t out_off[MAX_LAUNCH_LIMBS];  // per target: output limb (units of N)
    int32_t pid[MAX_LAUNCH_LIMBS];
};

// Precomputed launch maps (device copies) and their launch sizes.
struct MapRef {
    const LaunchMap* dev = nullptr;
    int n = 0;  // launch limbs (grid.y)
};
struct BcRef {
    const BcMap* dev = nullptr;
    int groups = 0;     // grid.y
    int n_in_max = 0;
};
struct KsPlan {             // key switching at one level (and rescale flag)
    MapRef up_rows, up_cols;  // ModUp INTT passes
    MapRef up_nrows;          // ModUp rows (not a digit's own) for an evaluation-domain row pass
    std::vector<BcRef> up_bc; // ModUp BConv + NTT column pass
    MapRef dn_cols;           // ModDown INTT column pass
    std::vector<BcRef> dn_bc; // ModDown BConv + NTT column pass
    MapRef dn_rows;           // ModDown NTT row pass + combine
};
struct RsPlan {             // stand-alone rescale at one level
    MapRef rows, cols, ncols, nrows;
};
struct RrPlan {             // stand-alone rational rescaling from a window to the window below
    MapRef rows, cols, nrows;     // INTT passes of the dropped rows; NTT row pass + combine
    std::vector<BcRef> bc;        // BConv dropped -> output primes + NTT column pass
};

// Item of a batched launch (device array written by the caller; same layout
// as ckks_batch_item in the C header).
struct BatchItem {
    int32_t level;   // operation level of this item
    int32_t key;     // index of its key in a key array (HRot), else 0
    int32_t rot;     // rotation k (HRot; Galois element 5^k mod 2N), else 0
    int32_t src;     // input slot this item reads (its output goes to slot i)
};

// Per-level directory of key-switch launch maps (device arrays of device
// pointers, indexed by level), used by batched launches.
struct KsDir {
    const LaunchMap* const* up_rows;
    const LaunchMap* const* up_cols;
    const BcMap* const* up_bc;
    const LaunchMap* const* dn_cols;
    const BcMap* const* dn_bc;
    const LaunchMap* const* dn_rows;
};

// Opt-in kernel timing (benchmarking only): while active, every kernel the
// library enqueues is bracketed by two hipEvents from a preallocated pool.
struct Profiler {
    bool active = false;
    int used = 0;
    std::vector<hipEvent_t> ev;           // 2 per launch
    std::vector<const char*> names;       // 1 per launch
    struct Agg {
        const char* name;
        int launches;
        double total_ms;
    };
    std::vector<Agg> agg;                 // filled by ckks_profile_kernels
};

struct Ctx {
    int device = 0;
    Profiler* prof = nullptr;
    int log_n = 0, n = 0;
    int n_q = 0, n_p = 0, dnum = 0, n_primes = 0;
    uint64_t mod[MAX_PRIMES] = {};  // host copy: q_0..q_{n_q-1}, p_0..p_{n_p-1}

    void* dev_block = nullptr;  // one allocation holding every table below
    size_t dev_bytes = 0;

    uint32_t* mods = nullptr;       // [n_primes]
    uint32_t* qinvs = nullptr;      // [n_primes] q^-1 mod 2^32
    // NTT twiddles: Shoup pairs (w, floor(w 2^32 / q))
    uint2* tw_fwd = nullptr;        // [n_primes][N] psi^brev(k)
    uint2* tw_inv = nullptr;        // [n_primes][N] psi^-brev(k)
    // the same twiddles as floor(w 2^32 / q) alone (w recovered in the kernel:
    // half the bytes; KeyMult's row passes)
    uint32_t* twq_fwd = nullptr;    // [n_primes][N]
    uint32_t* twq_inv = nullptr;    // [n_primes][N]
    // constants folded into the last inverse stage: (c, c_s, c w1, (c w1)_s),
    // w1 = psi^-brev(1) of the limb's prime, Shoup pairs
    uint4* ninv = nullptr;          // [n_primes] N^-1
    uint4* up_c_r = nullptr;        // [n_q+1][n_q] N^-1 [Dhat_{j,i}^-1]_{q_i} R, by level and prime id (input carries R^-1)
    uint4* up_c = nullptr;          // [n_q+1][n_q] N^-1 [Dhat_{j,i}^-1]_{q_i}
    int32_t* up_mat = nullptr;      // [n_q+1][dnum][n_primes][n_p] centred [Dhat_{j,s}]_t, by key digit
    uint4* dn_c = nullptr;          // [n_p + n_q] N^-1 [Phat_k^-1]_{p_k} R^2, then N^-1 R^2 [P^-1]_{q_i}
    int32_t* dn_mat = nullptr;      // [n_q][n_p] centred [Phat_k R^-1]_{q_i}
    uint2* dn_pinv = nullptr;       // [n_q] P^-1 R^2
    uint32_t* p_mod_q = nullptr;    // [n_q] [P]_{q_i} (plain residue, data operand)
    uint2* rinv = nullptr;          // [n_q] R^-1
    uint2* p_r2 = nullptr;          // [n_q] P R^-2
    uint2* r1 = nullptr;            // [n_q + n_p] R = 2^32 (undoes one Montgomery factor: PMult, plaintext weights)
    uint2* rs_qinv = nullptr;       // [n_q+1][n_q] [q_{l-1}^-1]_{q_i}
    int32_t* rs_mlast = nullptr;    // [n_q][n_p] centred [Phat_k P^-1 R]_{q_i}   (q_i the dropped prime)
    int32_t* rs_pr = nullptr;       // [n_q] centred [P R^-1]_{q_i}
    uint2* rs_fin = nullptr;        // [n_q+1][n_q] [P^-1 q_{l-1}^-1 R^2]_{q_i}
    // merged ModDown + rational rescaling (windowed contexts), S = P u D the
    // dropped primes, A the added ones, per level:
    uint4* rr_c = nullptr;          // N^-1 [Shat_s^-1]_s Q_A R^2 per s in S (INTT fold)
    int32_t* rr_mat = nullptr;      // centred [Shat_s R^-1 (Q_A^-1 if o is kept)]_o per (o, s)
    uint2* rr_fin = nullptr;        // [(Q_A if o is kept) Q_S^-1 R^2]_o per output row
    // stand-alone rational rescaling between a window and the window below
    // (S = D only; inputs carry no Montgomery factor): INTT fold
    // N^-1 [Dhat_d^-1]_d Q_A, matrix centred [Dhat_d R (Q_A^-1 if kept)]_o,
    // combine [(Q_A if kept) Q_D^-1]_o; offsets per level as above
    uint4* rr2_c = nullptr;
    int32_t* rr2_mat = nullptr;
    uint2* rr2_fin = nullptr;
    int rr2_c_off[MAX_PRIMES + 1] = {}, rr2_mat_off[MAX_PRIMES + 1] = {}, rr2_fin_off[MAX_PRIMES + 1] = {};
    // device copy of the per-level window data for batched launches (windowed
    // contexts): [4][MAX_PRIMES + 1] = wbase, rescaling's dropped rows (0: no
    // window below), rr_dlo, rr_dhi
    int32_t* lv_tab = nullptr;

    // launch plans, indexed by level (ks_plan[rescale][level], rs_plan[level])
    void* plan_block = nullptr;
    void* dir_block = nullptr;
    std::vector<KsPlan> ks_plan[2];
    std::vector<RsPlan> rs_plan;
    std::vector<RrPlan> rr_plan;   // windowed contexts, by level
    KsDir ks_dir[2] = {};  // per rescale flag; null entries where a level needs several BConv maps
    // tuning knobs (launch shapes only; results do not depend on them); the
    // defaults are the setting the tuner picks on MI355X at N = 2^16
    int tpw_up = 2;    // targets per work-group, ModUp BConv + NTT column pass (1, 2, 4)
    int tpw_dn = 2;    // the same for ModDown
    int xcd_pair = 1;  // column tiles of one 128-byte line on one XCD (0: tile = blockIdx.x)
    int rows_ept = 16; // residues per thread of the stand-alone row passes (16, or 4: one wave per row)
    int rows_ept1 = 4;  // the same for launches of a single operation (grid.z = 1)
    int km_ept = 4;     // residues per thread of KeyMult (16, or 4: one wave per row, k_keymult4)
    int km_ept1 = 4;    // the same for launches of a single operation
    int col_ept = 4;    // residues per thread of key switching's column passes (16, or 4: Col4 geometry)
    int col_ept1 = 4;   // the same for launches of a single operation
    int col_threads = 256;  // threads of a column-pass tile (256: 16 columns; 512: 32 columns = 128-byte rows)

    // Levels as windows of the prime list (Sec. 3.3): the level with `level`
    // limbs holds q_b .. q_{b+level-1}, b = wbase[level] (0 for every level of
    // a prefix context; -1 where a windowed context has no such level).  The
    // key's digits are fixed runs of n_p primes of the whole list (one key
    // over P * Q_max, Sec. 3.2); window digit j is the part of key digit
    // b / n_p + j inside the window, rows [digit_lo, digit_hi) of the window.
    int wbase[MAX_PRIMES + 1] = {};
    bool windowed = false;
    bool has_level(int level) const { return level >= 1 && level <= n_q && wbase[level] >= 0; }
    int woff(int level) const { return wbase[level] % n_p; }
    int digits(int level) const { return (woff(level) + level + n_p - 1) / n_p; }
    int key_digit(int j, int level) const { return wbase[level] / n_p + j; }
    int digit_lo(int j, int level) const { return j * n_p - woff(level) > 0 ? j * n_p - woff(level) : 0; }
    int digit_hi(int j, int level) const
    {
        return (j + 1) * n_p - woff(level) < level ? (j + 1) * n_p - woff(level) : level;
    }
    int row_pid(int r, int level) const { return r < level ? wbase[level] + r : n_q + (r - level); }

    // HMult + rescaling of a windowed context: ModDown merged into rational
    // rescaling to the window below (rr_below[level] limbs, 0 if none).  Rows
    // [rr_dlo, rr_dhi) of the window are kept (empty when rr_dhi <= rr_dlo);
    // the others are dropped with P.  The level's constants start at
    // rr_c_off (rows P then dropped), rr_mat_off ([below][n_p + dropped]) and
    // rr_fin_off (output rows) in rr_c / rr_mat / rr_fin.
    int rr_below[MAX_PRIMES + 1] = {};
    int rr_dlo[MAX_PRIMES + 1] = {}, rr_dhi[MAX_PRIMES + 1] = {};
    int rr_c_off[MAX_PRIMES + 1] = {}, rr_mat_off[MAX_PRIMES + 1] = {}, rr_fin_off[MAX_PRIMES + 1] = {};
    int rr_kept(int level) const { return rr_dhi[level] > rr_dlo[level] ? rr_dhi[level] - rr_dlo[level] : 0; }
    int rr_drop(int level) const { return level - rr_kept(level); }
    // output limbs of HMult + rescaling at `level` (0: none)
    int rs_out(int level) const { return windowed ? rr_below[level] : level - 1; }
    // rows rescaling takes to the coefficient domain besides P
    int rs_drop(int level) const { return windowed ? rr_drop(level) : 1; }
    // most rows a rescaling at a level up to `top` drops (workspace sizing)
    int rs_drop_max(int top) const
    {
        int d = 1;
        for (int l = 1; l <= top && windowed; l++)
            if (has_level(l) && rr_below[l] && rr_drop(l) > d) d = rr_drop(l);
        return d;
    }
};

// error reporting (thread-local message, see ckks_last_error)
int set_error(int code, const std::string& msg);
int check_hip(hipError_t e, const char* what);

// RAII bracket around one kernel launch (no-op unless profiling is active)
// Kernel timing while profiling: the launches inside a KTimer scope go
// through hipExtLaunchKernel with the scope's start / stop events, so the
// events carry the kernels' own start and end timestamps (the first launch
// sets start, every launch re-records stop).  A scope without a launch
// records both events at the same point.
struct KtEvents {
    hipEvent_t start = nullptr, stop = nullptr;
    bool started = false;
};
extern thread_local KtEvents* g_kt;
struct KTimer {
    Profiler* p;
    int slot = -1;
    hipStream_t s;
    KtEvents ev;
    KTimer(const Ctx& c, const char* name, hipStream_t st) : p(c.prof), s(st)
    {
        if (p && p->active && p->used < (int)p->names.size()) {
            slot = p->used++;
            p->names[slot] = name;
            ev.start = p->ev[2 * slot];
            ev.stop = p->ev[2 * slot + 1];
            g_kt = &ev;
        }
    }
    ~KTimer()
    {
        if (slot < 0) return;
        if (!ev.started) {
            (void)hipEventRecord(ev.start, s);
            (void)hipEventRecord(ev.stop, s);
        }
        g_kt = nullptr;
    }
};
// launch on `stream`, timed when a KTimer scope is open
#define CKKS_LAUNCH(K, GRID, BLOCK, SHMEM, STREAM, ...)                                                       \
    do {                                                                                                     \
        if (::ckks::g_kt) {                                                                                  \
            hipExtLaunchKernelGGL(K, GRID, BLOCK, SHMEM, STREAM, ::ckks::g_kt->started ? nullptr : ::ckks::g_kt->start, \
                                  ::ckks::g_kt->stop, 0, __VA_ARGS__);                                      \
            ::ckks::g_kt->started = true;                                                                    \
        } else {                                                                                             \
            hipLaunchKernelGGL(K, GRID, BLOCK, SHMEM, STREAM, __VA_ARGS__);                                  \
        }                                                                                                    \
    } while (0)

// ---------------------------------------------------------------------------
// launchers (kernels.hip).  All enqueue on `s` and return 0 or an error code.
// ---------------------------------------------------------------------------
// source of the digit's own rows; Hoisted also gathers the (evaluation-
// domain) ModUp rows instead of finishing their NTT
enum class Own { Tensor, Plain, Gather, Hoisted };
enum class Extra { None, HMult, HRot };     // term folded into ks before ModDown

struct KsIn {
    // HMult: a = (b_a, a_a), b = (b_b, a_b); KeySwitch: d; HRot: ct (b, a) + galois
    const uint32_t* b0 = nullptr;  // b_a | b (HRot) | -
    const uint32_t* a0 = nullptr;  // a_a | a (HRot) | d (KeySwitch)
    const uint32_t* b1 = nullptr;  // b_b
    const uint32_t* a1 = nullptr;  // a_b
    uint64_t galois = 1;
};

int launch_ntt(const Ctx& c, bool inverse, uint32_t* data, const int32_t* pids, int n_limbs, hipStream_t s);
int launch_bconv(const Ctx& c, const uint32_t* in, const int32_t* in_ids, int n_in, uint32_t* out,
                 const int32_t* out_ids, int n_out, void* ws, hipStream_t s);
// key switching core: writes ks (Q rows) to ks_q [2][level][N] and the lifted
// ModDown inputs; finishes with ModDown into out0 / out1.
// rescale = true (HMult only): also divide by q_{level-1} (rescale fused into
// ModDown); out0/out1 then have level-1 limbs.
int launch_keyswitch(const Ctx& c, Own own, Extra extra, const KsIn& in, int level, const uint32_t* evk,
                     uint32_t* out0, uint32_t* out1, void* ws, hipStream_t s, bool rescale = false);
int launch_rescale(const Ctx& c, const uint32_t* in, int level_in, uint32_t* out, void* ws, hipStream_t s);

// Batched key switching over n items with uniform per-item strides (residues):
// item i reads in.* + i*in_step (b1/a1: + i*in2_step), evk + key_i*key_step,
// writes out0/out1 + i*out_step, uses ws + i*ws_step; levels etc. from
// items[i] (device).  Grids are sized for max_level.
struct KsBatch {
    const BatchItem* items;
    int n, max_level;
    size_t in_step, in2_step, out_step, ws_step, key_step;
    int n_keys;  // valid key indices [0, n_keys) (1 when every item uses the same key)
    int n_src;   // valid input slots [0, n_src)
};
int launch_hrot_hoisted(const Ctx& c, const uint32_t* b_in, const uint32_t* a_in, int level, int n_rot,
                        const BatchItem* items, const uint32_t* keys, int n_keys, size_t key_step, uint32_t* outs,
                        void* ws, hipStream_t s);
int launch_hrot_sum_hoisted(const Ctx& c, const uint32_t* b_in, const uint32_t* a_in, int level, int n_rot,
                            const BatchItem* items, const uint32_t* keys, int n_keys, size_t key_step,
                            const uint32_t* pts, size_t pt_step, uint32_t* out, void* ws, hipStream_t s);
int launch_keyswitch_batch(const Ctx& c, Own own, Extra extra, const KsIn& in, const KsBatch& b,
                           const uint32_t* evk, uint32_t* out0, uint32_t* out1, void* ws, hipStream_t s,
                           bool rescale);

// element-wise mechanisms (elementwise.hip): out[h][i] = op(a[h][i], b[h or -][i])
enum class Ew { HAdd, PAdd, PMult };
int launch_elementwise(const Ctx& c, Ew op, const uint32_t* a, int level_a, const uint32_t* b, int level_b,
                       int level, uint32_t* out, hipStream_t s);

// out[h][l] = a_l * x[h][xrow_l] + b_l * y[h][l]  (mod the limb's prime; a term
// is absent when xrow_l < 0 or y is null); constants twisted (mulc)
struct LincombArgs {
    int n;                      // limbs
    int32_t xrow[MAX_PRIMES];   // row of x feeding limb l, or -1
    uint32_t q[MAX_PRIMES];
    uint2 a[MAX_PRIMES], b[MAX_PRIMES];
};
int launch_lincomb(const Ctx& c, const LincombArgs& L, const uint32_t* x, size_t x_half, const uint32_t* y,
                   size_t y_half, uint32_t* out, size_t o_half, hipStream_t s);
// rational rescaling between two prime sets (ids into the context's primes)
int launch_rescale_rational_window(const Ctx& c, int level, const uint32_t* ct, uint32_t* out, void* ws,
                                   hipStream_t s);
int launch_rescale_rational(const Ctx& c, const uint32_t* ct, int n_in, const int32_t* in_ids, int n_out,
                            const int32_t* out_ids, uint32_t* out, void* ws, hipStream_t s);
size_t rescale_rational_ws_bytes(const Ctx& c, int n_in, int n_out);
// host copy of the stand-alone base conversion's constants (ctx.cpp)
void bconv_consts(const Ctx& c, const int32_t* in_ids, int n_in, const int32_t* out_ids, int n_out, uint2* cs,
                  int32_t* ms);

// builds every launch plan and uploads the maps (context creation)
int build_plans(Ctx& c);
// sets the tuning knobs and rebuilds the plans
int retune(Ctx& c, int tpw_up, int tpw_dn, int xcd_pair, int rows_ept, int rows_ept1, int col_threads, int km_ept,
           int km_ept1, int col_ept, int col_ept1);

size_t keyswitch_ws_bytes(const Ctx& c, int level);
size_t rescale_ws_bytes(const Ctx& c);
size_t bconv_ws_bytes(const Ctx& c, int n_in, int n_out);

}  // namespace ckks
