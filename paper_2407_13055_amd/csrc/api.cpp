// C-ABI entry points: argument validation, then the launch sequences of
// kernels.hip.  Nothing here computes on residues.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>

#include "../../include/ckks_hip.h"
#include "internal.h"

struct ckks_ctx {
    ckks::Ctx* impl;
};

// Workspace of ckks_hmult_rescale_noalloc: one array per GPU, placed by the
// code-object loader.  In host code `scratch` names a host-side stand-in, so
// its device address is looked up once per GPU (scratch_setup, at context
// creation with that GPU current) and only that address is used.
static __device__ __align__(256) uint8_t scratch[CKKS_NOALLOC_SCRATCH_BYTES];

namespace ckks {

int build_ctx(const ckks_params* p, const int32_t* win_start, const int32_t* win_len, int n_win, Ctx** out);
void free_ctx(Ctx* c);
int prime_chain(int bits, int log_n, int count, uint64_t* out);

static thread_local std::string g_last_error;

int set_error(int code, const std::string& msg)
{
    g_last_error = msg;
    return code;
}

int check_hip(hipError_t e, const char* what)
{
    if (e == hipSuccess) return 0;
    return set_error(CKKS_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

namespace {

int check_ctx(const ckks_ctx* ctx)
{
    if (!ctx || !ctx->impl) return set_error(CKKS_EINVAL, "null context");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return set_error(CKKS_EHIP, "hipGetDevice failed");
    if (dev != ctx->impl->device) return set_error(CKKS_EINVAL, "current device differs from the context's device");
    return 0;
}

int check_ptr(const void* p, const char* name)
{
    if (!p) return set_error(CKKS_EINVAL, std::string("null pointer: ") + name);
    if (reinterpret_cast<uintptr_t>(p) % 16) return set_error(CKKS_EALIGN, std::string("misaligned pointer: ") + name);
    return 0;
}

int check_ws(const void* ws, size_t have, size_t need)
{
    if (need && (!ws || have < need))
        return set_error(CKKS_EWORKSPACE, "workspace smaller than ckks_workspace_size reports (" + std::to_string(need) +
                                              " bytes)");
    if (ws && reinterpret_cast<uintptr_t>(ws) % 16) return set_error(CKKS_EALIGN, "misaligned workspace");
    return 0;
}

// [a, a + na) and [b, b + nb) in residues
bool overlap(const void* a, size_t na, const void* b, size_t nb)
{
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y + nb * 4 && y < x + na * 4;
}

int check_level(const Ctx& c, int level, int lo)
{
    if (level < lo || level > c.n_q) return set_error(CKKS_EINVAL, "level out of range");
    if (!c.has_level(level)) return set_error(CKKS_EINVAL, "the context has no level with this many limbs");
    return 0;
}

// Inputs of a prefix context may sit at a higher level (the first `level`
// limbs are used); a windowed context's levels are not prefixes of each
// other, so its inputs must be at the operation level.
int check_in(const Ctx& c, int level_in, int level)
{
    if (level_in < level || level_in > c.n_q) return set_error(CKKS_EINVAL, "input level below the operation level");
    if (c.windowed && level_in != level)
        return set_error(CKKS_EINVAL, "a windowed context takes inputs at exactly the operation level");
    return 0;
}

// Single rescaling by the last prime runs on prefix contexts only (a
// windowed context rescales rationally between windows).
int check_prefix(const Ctx& c, const char* what)
{
    if (c.windowed) return set_error(CKKS_EUNSUPPORTED, std::string(what) + " is not available on a windowed context");
    return 0;
}

hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

constexpr int kMaxDevices = 256;
std::mutex g_scratch_mu;
std::atomic<void*> g_scratch_ptr[kMaxDevices];

// Device address of `scratch` on `device` (the current device), looked up
// on the first call for that device.
int scratch_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return set_error(CKKS_EUNSUPPORTED, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device].load()) return 0;
    void* p = nullptr;
    if (int e = check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)")) return e;
    if (!p) return set_error(CKKS_EHIP, "hipGetSymbolAddress(scratch) returned a null address");
    g_scratch_ptr[device].store(p);
    return 0;
}

}  // namespace
}  // namespace ckks

using namespace ckks;

extern "C" {

const char* ckks_last_error(void) { return g_last_error.c_str(); }

int ckks_prime_chain(int bits, int log_n, int count, uint64_t* out) { return prime_chain(bits, log_n, count, out); }

int ckks_ctx_create(const ckks_params* params, ckks_ctx** out)
{
    if (!out) return set_error(CKKS_EINVAL, "null output pointer");
    Ctx* c = nullptr;
    if (int e = build_ctx(params, nullptr, nullptr, 0, &c)) return e;
    if (int e = scratch_setup(c->device)) {
        free_ctx(c);
        return e;
    }
    *out = new ckks_ctx{c};
    return CKKS_OK;
}

int ckks_ctx_create_windowed(const ckks_params* params, const int32_t* win_start, const int32_t* win_len, int n_win,
                             ckks_ctx** out)
{
    if (!out) return set_error(CKKS_EINVAL, "null output pointer");
    if (!win_start || !win_len) return set_error(CKKS_EINVAL, "null window array");
    Ctx* c = nullptr;
    if (int e = build_ctx(params, win_start, win_len, n_win, &c)) return e;
    if (int e = scratch_setup(c->device)) {
        free_ctx(c);
        return e;
    }
    *out = new ckks_ctx{c};
    return CKKS_OK;
}

static void free_profiler(Ctx* c)
{
    if (!c || !c->prof) return;
    for (hipEvent_t e : c->prof->ev) (void)hipEventDestroy(e);
    delete c->prof;
    c->prof = nullptr;
}

void ckks_ctx_destroy(ckks_ctx* ctx)
{
    if (!ctx) return;
    free_profiler(ctx->impl);
    free_ctx(ctx->impl);
    delete ctx;
}

int ckks_ctx_tune(ckks_ctx* ctx, const ckks_tuning* t)
{
    if (int e = check_ctx(ctx)) return e;
    if (!t) return set_error(CKKS_EINVAL, "null tuning");
    auto tpw_ok = [](int v) { return v == 1 || v == 2 || v == 4; };
    if (!tpw_ok(t->bconv_tpw_up) || !tpw_ok(t->bconv_tpw_down))
        return set_error(CKKS_EINVAL, "bconv targets per work-group must be 1, 2 or 4");
    if (t->xcd_pair != 0 && t->xcd_pair != 1) return set_error(CKKS_EINVAL, "xcd_pair must be 0 or 1");
    if (t->rows_per_thread != 4 && t->rows_per_thread != 16)
        return set_error(CKKS_EINVAL, "rows_per_thread must be 4 or 16");
    if (t->col_threads != 128 && t->col_threads != 256 && t->col_threads != 512)
        return set_error(CKKS_EINVAL, "col_threads must be 128, 256 or 512");
    if (t->rows_per_thread_single != 0 && t->rows_per_thread_single != 4 && t->rows_per_thread_single != 16)
        return set_error(CKKS_EINVAL, "rows_per_thread_single must be 0, 4 or 16");
    if (t->keymult_rows != 4 && t->keymult_rows != 16) return set_error(CKKS_EINVAL, "keymult_rows must be 4 or 16");
    if (t->keymult_rows_single != 0 && t->keymult_rows_single != 4 && t->keymult_rows_single != 16)
        return set_error(CKKS_EINVAL, "keymult_rows_single must be 0, 4 or 16");
    if (t->cols_per_thread != 4 && t->cols_per_thread != 16)
        return set_error(CKKS_EINVAL, "cols_per_thread must be 4 or 16");
    if (t->cols_per_thread_single != 0 && t->cols_per_thread_single != 4 && t->cols_per_thread_single != 16)
        return set_error(CKKS_EINVAL, "cols_per_thread_single must be 0, 4 or 16");
    if (int e = check_hip(hipDeviceSynchronize(), "synchronize before retuning")) return e;
    return retune(*ctx->impl, t->bconv_tpw_up, t->bconv_tpw_down, t->xcd_pair, t->rows_per_thread,
                  t->rows_per_thread_single ? t->rows_per_thread_single : t->rows_per_thread, t->col_threads,
                  t->keymult_rows, t->keymult_rows_single ? t->keymult_rows_single : t->keymult_rows,
                  t->cols_per_thread, t->cols_per_thread_single ? t->cols_per_thread_single : t->cols_per_thread);
}

int ckks_ctx_tuning(const ckks_ctx* ctx, ckks_tuning* out)
{
    if (!ctx || !ctx->impl || !out) return set_error(CKKS_EINVAL, "null argument");
    const Ctx& c = *ctx->impl;
    out->bconv_tpw_up = c.tpw_up;
    out->bconv_tpw_down = c.tpw_dn;
    out->xcd_pair = c.xcd_pair;
    out->rows_per_thread = c.rows_ept;
    out->col_threads = c.col_threads;
    out->rows_per_thread_single = c.rows_ept1;
    out->keymult_rows = c.km_ept;
    out->keymult_rows_single = c.km_ept1;
    out->cols_per_thread = c.col_ept;
    out->cols_per_thread_single = c.col_ept1;
    return CKKS_OK;
}

int ckks_profile_start(ckks_ctx* ctx, int max_launches)
{
    if (int e = check_ctx(ctx)) return e;
    if (max_launches < 1 || max_launches > (1 << 20)) return set_error(CKKS_EINVAL, "bad max_launches");
    Ctx& c = *ctx->impl;
    if (!c.prof || (int)c.prof->names.size() < max_launches) {
        free_profiler(&c);
        c.prof = new Profiler();
        c.prof->names.assign(max_launches, nullptr);
        c.prof->ev.assign(2 * (size_t)max_launches, nullptr);
        for (auto& e : c.prof->ev)
            if (hipEventCreate(&e) != hipSuccess) {
                free_profiler(&c);
                return set_error(CKKS_EHIP, "hipEventCreate failed");
            }
    }
    c.prof->used = 0;
    c.prof->agg.clear();
    c.prof->active = true;
    return CKKS_OK;
}

int ckks_profile_stop(ckks_ctx* ctx)
{
    if (int e = check_ctx(ctx)) return e;
    if (ctx->impl->prof) ctx->impl->prof->active = false;
    return CKKS_OK;
}

int ckks_profile_kernels(ckks_ctx* ctx, int* n_kernels)
{
    if (int e = check_ctx(ctx)) return e;
    if (!n_kernels) return set_error(CKKS_EINVAL, "null output");
    Profiler* p = ctx->impl->prof;
    *n_kernels = 0;
    if (!p) return CKKS_OK;
    p->agg.clear();
    for (int i = 0; i < p->used; i++) {
        if (hipEventSynchronize(p->ev[2 * i + 1]) != hipSuccess) return set_error(CKKS_EHIP, "event sync failed");
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p->ev[2 * i], p->ev[2 * i + 1]) != hipSuccess)
            return set_error(CKKS_EHIP, "event elapsed time failed");
        bool found = false;
        for (auto& a : p->agg)
            if (std::strcmp(a.name, p->names[i]) == 0) {
                a.launches++, a.total_ms += ms, found = true;
                break;
            }
        if (!found) p->agg.push_back({p->names[i], 1, (double)ms});
    }
    *n_kernels = (int)p->agg.size();
    return CKKS_OK;
}

int ckks_profile_kernel(ckks_ctx* ctx, int i, const char** name, int* launches, double* total_ms)
{
    if (int e = check_ctx(ctx)) return e;
    Profiler* p = ctx->impl->prof;
    if (!p || i < 0 || i >= (int)p->agg.size() || !name || !launches || !total_ms)
        return set_error(CKKS_EINVAL, "bad profile query");
    *name = p->agg[i].name;
    *launches = p->agg[i].launches;
    *total_ms = p->agg[i].total_ms;
    return CKKS_OK;
}

int ckks_workspace_size(const ckks_ctx* ctx, int op, int level, int n_in, int n_out, size_t* bytes)
{
    if (!ctx || !ctx->impl || !bytes) return set_error(CKKS_EINVAL, "null argument");
    const Ctx& c = *ctx->impl;
    switch (op) {
    case CKKS_OP_BCONV:
        if (n_in < 1 || n_out < 1 || n_in > MAX_PRIMES || n_out > MAX_PRIMES)
            return set_error(CKKS_EINVAL, "bad bconv sizes");
        *bytes = bconv_ws_bytes(c, n_in, n_out);
        return CKKS_OK;
    case CKKS_OP_KEYSWITCH:
    case CKKS_OP_HMULT:
    case CKKS_OP_HROT:
        if (int e = check_level(c, level, 1)) return e;
        *bytes = keyswitch_ws_bytes(c, level);
        return CKKS_OK;
    case CKKS_OP_RESCALE:
        *bytes = rescale_ws_bytes(c);
        return CKKS_OK;
    case CKKS_OP_HROT_HOISTED:  /* n_in = number of rotations */
        if (int e = check_level(c, level, 1)) return e;
        if (n_in < 1) return set_error(CKKS_EINVAL, "rotation count must be >= 1");
        *bytes = keyswitch_ws_bytes(c, level) * ((size_t)n_in + 1);
        return CKKS_OK;
    case CKKS_OP_RESCALE_RATIONAL:  /* n_in input limbs, n_out output limbs */
        if (n_in < 1 || n_out < 1 || n_in > MAX_PRIMES || n_out > MAX_PRIMES)
            return set_error(CKKS_EINVAL, "bad limb counts");
        *bytes = rescale_rational_ws_bytes(c, n_in, n_out);
        return CKKS_OK;
    case CKKS_OP_HROT_SUM:  /* any number of rotations */
        if (int e = check_level(c, level, 1)) return e;
        *bytes = 2 * keyswitch_ws_bytes(c, level);
        return CKKS_OK;
    default:
        return set_error(CKKS_EINVAL, "unknown op");
    }
}

static int ntt_common(const ckks_ctx* ctx, uint32_t* data, const int32_t* ids, int n_limbs, void* stream, bool inv)
{
    if (int e = check_ctx(ctx)) return e;
    const Ctx& c = *ctx->impl;
    if (n_limbs < 0 || (n_limbs && !ids)) return set_error(CKKS_EINVAL, "bad limb list");
    if (n_limbs == 0) return CKKS_OK;
    if (int e = check_ptr(data, "data")) return e;
    for (int i = 0; i < n_limbs; i++)
        if (ids[i] < 0 || ids[i] >= c.n_primes) return set_error(CKKS_EINVAL, "prime id out of range");
    return launch_ntt(c, inv, data, ids, n_limbs, as_stream(stream));
}

int ckks_ntt(const ckks_ctx* ctx, uint32_t* data, const int32_t* prime_ids, int n_limbs, void* stream)
{
    return ntt_common(ctx, data, prime_ids, n_limbs, stream, false);
}

int ckks_intt(const ckks_ctx* ctx, uint32_t* data, const int32_t* prime_ids, int n_limbs, void* stream)
{
    return ntt_common(ctx, data, prime_ids, n_limbs, stream, true);
}

int ckks_bconv(const ckks_ctx* ctx, const uint32_t* in, const int32_t* in_ids, int n_in, uint32_t* out,
               const int32_t* out_ids, int n_out, void* ws, size_t ws_bytes, void* stream)
{
    if (int e = check_ctx(ctx)) return e;
    const Ctx& c = *ctx->impl;
    if (n_in < 1 || n_out < 1 || n_in > MAX_PRIMES || n_out > MAX_PRIMES || !in_ids || !out_ids)
        return set_error(CKKS_EINVAL, "bad bconv sizes");
    if (int e = check_ptr(in, "in")) return e;
    if (int e = check_ptr(out, "out")) return e;
    for (int i = 0; i < n_in; i++) {
        if (in_ids[i] < 0 || in_ids[i] >= c.n_primes) return set_error(CKKS_EINVAL, "prime id out of range");
        for (int k = 0; k < i; k++)
            if (in_ids[k] == in_ids[i]) return set_error(CKKS_EINVAL, "input primes must be distinct");
    }
    for (int i = 0; i < n_out; i++)
        if (out_ids[i] < 0 || out_ids[i] >= c.n_primes) return set_error(CKKS_EINVAL, "prime id out of range");
    if (overlap(in, (size_t)n_in * c.n, out, (size_t)n_out * c.n)) return set_error(CKKS_EINVAL, "out overlaps in");
    if (int e = check_ws(ws, ws_bytes, bconv_ws_bytes(c, n_in, n_out))) return e;
    return launch_bconv(c, in, in_ids, n_in, out, out_ids, n_out, ws, as_stream(stream));
}

int ckks_keyswitch(const ckks_ctx* ctx, const uint32_t* d, int level, const uint32_t* evk, uint32_t* out0,
                   uint32_t* out1, void* ws, size_t ws_bytes, void* stream)
{
    if (int e = check_ctx(ctx)) return e;
    const Ctx& c = *ctx->impl;
    if (int e = check_level(c, level, 1)) return e;
    for (auto [p, nm] : {std::pair<const void*, const char*>{d, "d"}, {evk, "evk"}, {out0, "out0"}, {out1, "out1"}})
        if (int e = check_ptr(p, nm)) return e;
    const size_t L = (size_t)level * c.n;
    if (overlap(out0, L, out1, L) || overlap(out0, L, d, L) || overlap(out1, L, d, L))
        return set_error(CKKS_EINVAL, "outputs overlap");
    if (int e = check_ws(ws, ws_bytes, keyswitch_ws_bytes(c, level))) return e;
    KsIn in;
    in.a0 = d;
    return launch_keyswitch(c, Own::Plain, Extra::None, in, level, evk, out0, out1, ws, as_stream(stream));
}

int ckks_hmult(const ckks_ctx* ctx, const uint32_t* ct_a, int level_a, const uint32_t* ct_b, int level_b,
               const uint32_t* rlk, int level, uint32_t* out, void* ws, size_t ws_bytes, void* stream)
{
    if (int e = check_ctx(ctx)) return e;
    const Ctx& c = *ctx->impl;
    if (int e = check_level(c, level, 1)) return e;
    if (int e = check_in(c, level_a, level)) return e;
    if (int e = check_in(c, level_b, level)) return e;
    for (auto [p, nm] : {std::pair<const void*, const char*>{ct_a, "ct_a"}, {ct_b, "ct_b"}, {rlk, "rlk"}, {out, "out"}})
        if (int e = check_ptr(p, nm)) return e;
    const size_t n = c.n;
    if (overlap(out, 2 * level * n, ct_a, 2 * level_a * n) || overlap(out, 2 * level * n, ct_b, 2 * level_b * n))
        return set_error(CKKS_EINVAL, "out overlaps an input");
    if (int e = check_ws(ws, ws_bytes, keyswitch_ws_bytes(c, level))) return e;
    KsIn in;
    in.b0 = ct_a;
    in.a0 = ct_a + (size_t)level_a * n;
    in.b1 = ct_b;
    in.a1 = ct_b + (size_t)level_b * n;
    return launch_keyswitch(c, Own::Tensor, Extra::HMult, in, level, rlk, out, out + (size_t)level * n, ws,
                            as_stream(stream));
}

static int hmult_rescale_checked(const ckks_ctx* ctx, const uint32_t* ct_a, int level_a, const uint32_t* ct_b,
                                 int level_b, const uint32_t* rlk, int level, uint32_t* out, void* ws,
                                 size_t ws_bytes, void* stream)
{
    const Ctx& c = *ctx->impl;
    if (int e = check_level(c, level, c.windowed ? 1 : 2)) return e;
    if (c.rs_out(level) < 1) return set_error(CKKS_EINVAL, "no level below this one to rescale to");
    if (int e = check_in(c, level_a, level)) return e;
    if (int e = check_in(c, level_b, level)) return e;
    for (auto [p, nm] : {std::pair<const void*, const char*>{ct_a, "ct_a"}, {ct_b, "ct_b"}, {rlk, "rlk"}, {out, "out"}})
        if (int e = check_ptr(p, nm)) return e;
    const size_t n = c.n, lo = (size_t)c.rs_out(level);
    if (overlap(out, 2 * lo * n, ct_a, 2 * level_a * n) || overlap(out, 2 * lo * n, ct_b, 2 * level_b * n))
        return set_error(CKKS_EINVAL, "out overlaps an input");
    if (int e = check_ws(ws, ws_bytes, keyswitch_ws_bytes(c, level))) return e;
    KsIn in;
    in.b0 = ct_a;
    in.a0 = ct_a + (size_t)level_a * n;
    in.b1 = ct_b;
    in.a1 = ct_b + (size_t)level_b * n;
    return launch_keyswitch(c, Own::Tensor, Extra::HMult, in, level, rlk, out, out + lo * n, ws, as_stream(stream),
                            true);
}

int ckks_hmult_rescale(const ckks_ctx* ctx, const uint32_t* ct_a, int level_a, const uint32_t* ct_b, int level_b,
                       const uint32_t* rlk, int level, uint32_t* out, void* ws, size_t ws_bytes, void* stream)
{
    if (int e = check_ctx(ctx)) return e;
    return hmult_rescale_checked(ctx, ct_a, level_a, ct_b, level_b, rlk, level, out, ws, ws_bytes, stream);
}

int ckks_hmult_rescale_noalloc(const ckks_ctx* ctx, const uint32_t* ct_a, int level_a, const uint32_t* ct_b,
                               int level_b, const uint32_t* rlk, int level, uint32_t* out, void* stream)
{
    if (int e = check_ctx(ctx)) return e;
    const Ctx& c = *ctx->impl;
    if (int e = check_level(c, level, c.windowed ? 1 : 2)) return e;
    const size_t need = keyswitch_ws_bytes(c, level);
    if (need > CKKS_NOALLOC_SCRATCH_BYTES)
        return set_error(CKKS_EWORKSPACE, "this level needs " + std::to_string(need) +
                                              " workspace bytes; the allocation-free call holds " +
                                              std::to_string((size_t)CKKS_NOALLOC_SCRATCH_BYTES));
    void* ws = g_scratch_ptr[c.device].load();
    if (!ws) return set_error(CKKS_EHIP, "no scratch address for this device");
    return hmult_rescale_checked(ctx, ct_a, level_a, ct_b, level_b, rlk, level, out, ws,
                                 CKKS_NOALLOC_SCRATCH_BYTES, stream);
}

static int hmult_batch(const ckks_ctx* ctx, int n, const uint32_t* a, const uint32_t* b, int n_src, int level_in,
                       const ckks_batch_item* items, int max_level, const uint32_t* rlk, uint32_t* out, void* ws,
                       size_t ws_bytes, void* stream, bool rescale)
{
    if (int e = check_ctx(ctx)) return e;
    const Ctx& c = *ctx->impl;
    if (n < 1 || n > 65535) return set_error(CKKS_EINVAL, "batch size out of range");
    if (n_src < 1) return set_error(CKKS_EINVAL, "need at least one input slot");
    if (int e = check_level(c, max_level, rescale && !c.windowed ? 2 : 1)) return e;
    if (rescale && c.rs_out(max_level) < 1) return set_error(CKKS_EINVAL, "no level below max_level to rescale to");
    if (level_in < max_level || level_in > c.n_q) return set_error(CKKS_EINVAL, "level_in below max_level");
    for (auto [p, nm] : {std::pair<const void*, const char*>{a, "a"}, {b, "b"}, {items, "items"}, {rlk, "rlk"},
                         {out, "out"}})
        if (int e = check_ptr(p, nm)) return e;
    const int out_level = rescale ? c.rs_out(max_level) : max_level;
    const size_t N = c.n, in_step = 2 * (size_t)level_in * N, out_step = 2 * (size_t)out_level * N;
    if (overlap(out, n * out_step, a, n_src * in_step) || overlap(out, n * out_step, b, n_src * in_step))
        return set_error(CKKS_EINVAL, "out overlaps an input");
    const size_t per = keyswitch_ws_bytes(c, max_level);
    if (int e = check_ws(ws, ws_bytes, per * (size_t)n)) return e;
    KsIn in;
    in.b0 = a;
    in.a0 = a + (size_t)level_in * N;
    in.b1 = b;
    in.a1 = b + (size_t)level_in * N;
    KsBatch bt{reinterpret_cast<const BatchItem*>(items), n, max_level, in_step, in_step, out_step, per / 4, 0, 1, n_src};
    return launch_keyswitch_batch(c, Own::Tensor, Extra::HMult, in, bt, rlk, out, out + (size_t)out_level * N, ws,
                                  as_stream(stream), rescale);
}

int ckks_hmult_batch(const ckks_ctx* ctx, int n, const uint32_t* a, const uint32_t* b, int n_src, int level_in,
                     const ckks_batch_item* items, int max_level, const uint32_t* rlk, uint32_t* out, void* ws,
                     size_t ws_bytes, void* stream)
{
    return hmult_batch(ctx, n, a, b, n_src, level_in, items, max_level, rlk, out, ws, ws_bytes, stream, false);
}

int ckks_hmult_rescale_batch(const ckks_ctx* ctx, int n, const uint32_t* a, const uint32_t* b, int n_src, int level_in,
                             const ckks_batch_item* items, int max_level, const uint32_t* rlk, uint32_t* out,
                             void* ws, size_t ws_bytes, void* stream)
{
    return hmult_batch(ctx, n, a, b, n_src, level_in, items, max_level, rlk, out, ws, ws_bytes, stream, true);
}

int ckks_hrot_batch(const ckks_ctx* ctx, int n, const uint32_t* ct, int n_src, int level_in,
                    const ckks_batch_item* items, int max_level, const uint32_t* keys, int n_keys, uint32_t* out,
                    void* ws, size_t ws_bytes, void* stream)
{
    if (int e = check_ctx(ctx)) return e;
    const Ctx& c = *ctx->impl;
    if (n < 1 || n > 65535) return set_error(CKKS_EINVAL, "batch size out of range");
    if (n_src < 1) return set_error(CKKS_EINVAL, "need at least one input slot");
    if (n_keys < 1) return set_error(CKKS_EINVAL, "need at least one key");
    if (int e = check_level(c, max_level, 1)) return e;
    if (level_in < max_level || level_in > c.n_q) return set_error(CKKS_EINVAL, "level_in below max_level");
    for (auto [p, nm] : {std::pair<const void*, const char*>{ct, "ct"}, {items, "items"}, {keys, "keys"}, {out, "out"}})
        if (int e = check_ptr(p, nm)) return e;
    const size_t N = c.n, in_step = 2 * (size_t)level_in * N, out_step = 2 * (size_t)max_level * N;
    if (overlap(out, n * out_step, ct, n_src * in_step)) return set_error(CKKS_EINVAL, "out overlaps the input");
    const size_t per = keyswitch_ws_bytes(c, max_level);
    if (int e = check_ws(ws, ws_bytes, per * (size_t)n)) return e;
    KsIn in;
    in.b0 = ct;
    in.a0 = ct + (size_t)level_in * N;
    const size_t key_step = (size_t)c.dnum * 2 * (c.n_q + c.n_p) * N;
    KsBatch bt{reinterpret_cast<const BatchItem*>(items), n, max_level, in_step, 0, out_step, per / 4, key_step, n_keys,
               n_src};
    return launch_keyswitch_batch(c, Own::Gather, Extra::HRot, in, bt, keys, out, out + (size_t)max_level * N, ws,
                                  as_stream(stream), false);
}

int ckks_hrot_hoisted(const ckks_ctx* ctx, const uint32_t* ct, int level_in, int level, int n_rot,
                      const ckks_batch_item* items, const uint32_t* keys, int n_keys, uint32_t* outs, void* ws,
                      size_t ws_bytes, void* stream)
{
    if (int e = check_ctx(ctx)) return e;
    const Ctx& c = *ctx->impl;
    if (n_rot < 1 || n_rot > 65535) return set_error(CKKS_EINVAL, "rotation count out of range");
    if (n_keys < 1) return set_error(CKKS_EINVAL, "need at least one key");
    if (int e = check_level(c, level, 1)) return e;
    if (int e = check_in(c, level_in, level)) return e;
    for (auto [p, nm] : {std::pair<const void*, const char*>{ct, "ct"}, {items, "items"}, {keys, "keys"}, {outs, "outs"}})
        if (int e = check_ptr(p, nm)) return e;
    const size_t N = c.n;
    if (overlap(outs, (size_t)n_rot * 2 * level * N, ct, 2 * (size_t)level_in * N))
        return set_error(CKKS_EINVAL, "outs overlap the input");
    if (int e = check_ws(ws, ws_bytes, keyswitch_ws_bytes(c, level) * ((size_t)n_rot + 1))) return e;
    const size_t key_step = (size_t)c.dnum * 2 * (c.n_q + c.n_p) * N;
    return launch_hrot_hoisted(c, ct, ct + (size_t)level_in * N, level, n_rot, reinterpret_cast<const BatchItem*>(items),
                               keys, n_keys, key_step, outs, ws, as_stream(stream));
}

int ckks_hrot_sum_hoisted(const ckks_ctx* ctx, const uint32_t* ct, int level_in, int level, int n_rot,
                          const ckks_batch_item* items, const uint32_t* keys, int n_keys, const uint32_t* pts,
                          uint32_t* out, void* ws, size_t ws_bytes, void* stream)
{
    if (int e = check_ctx(ctx)) return e;
    const Ctx& c = *ctx->impl;
    if (n_rot < 1 || n_rot > 65535) return set_error(CKKS_EINVAL, "rotation count out of range");
    if (n_keys < 1) return set_error(CKKS_EINVAL, "need at least one key");
    if (int e = check_level(c, level, 1)) return e;
    if (int e = check_in(c, level_in, level)) return e;
    for (auto [p, nm] : {std::pair<const void*, const char*>{ct, "ct"}, {items, "items"}, {keys, "keys"},
                         {pts, "pts"}, {out, "out"}})
        if (int e = check_ptr(p, nm)) return e;
    const size_t N = c.n, pt_step = (size_t)(c.n_q + c.n_p) * N;
    if (overlap(out, 2 * (size_t)level * N, ct, 2 * (size_t)level_in * N) ||
        overlap(out, 2 * (size_t)level * N, pts, (size_t)n_rot * pt_step))
        return set_error(CKKS_EINVAL, "out overlaps an input");
    if (int e = check_ws(ws, ws_bytes, 2 * keyswitch_ws_bytes(c, level))) return e;
    const size_t key_step = (size_t)c.dnum * 2 * (c.n_q + c.n_p) * N;
    return launch_hrot_sum_hoisted(c, ct, ct + (size_t)level_in * N, level, n_rot,
                                   reinterpret_cast<const BatchItem*>(items), keys, n_keys, key_step, pts, pt_step,
                                   out, ws, as_stream(stream));
}

int ckks_hrot(const ckks_ctx* ctx, const uint32_t* ct, int level_in, int level, int k, const uint32_t* rk,
              uint32_t* out, void* ws, size_t ws_bytes, void* stream)
{
    if (int e = check_ctx(ctx)) return e;
    const Ctx& c = *ctx->impl;
    if (int e = check_level(c, level, 1)) return e;
    if (int e = check_in(c, level_in, level)) return e;
    for (auto [p, nm] : {std::pair<const void*, const char*>{ct, "ct"}, {rk, "rk"}, {out, "out"}})
        if (int e = check_ptr(p, nm)) return e;
    const size_t n = c.n;
    if (overlap(out, 2 * level * n, ct, 2 * level_in * n)) return set_error(CKKS_EINVAL, "out overlaps the input");
    if (int e = check_ws(ws, ws_bytes, keyswitch_ws_bytes(c, level))) return e;
    const uint64_t two_n = 2ull * c.n, half = (uint64_t)c.n / 2;
    const uint64_t kk = (uint64_t)(((int64_t)k % (int64_t)half + (int64_t)half) % (int64_t)half);
    uint64_t g = 1, b = 5;
    for (uint64_t e = kk; e; e >>= 1, b = b * b % two_n)
        if (e & 1) g = g * b % two_n;
    KsIn in;
    in.b0 = ct;
    in.a0 = ct + (size_t)level_in * n;
    in.galois = g;
    return launch_keyswitch(c, Own::Gather, Extra::HRot, in, level, rk, out, out + (size_t)level * n, ws,
                            as_stream(stream));
}

// out may equal an input exactly (in place); partial overlap is rejected
static int elementwise(const ckks_ctx* ctx, Ew op, const uint32_t* a, int level_a, const uint32_t* b, int b_limbs,
                       int level, uint32_t* out, void* stream)
{
    if (int e = check_ctx(ctx)) return e;
    const Ctx& c = *ctx->impl;
    if (int e = check_level(c, level, 1)) return e;
    if (int e = check_in(c, level_a, level)) return e;
    const int b_max = op == Ew::HAdd ? c.n_q : c.n_q + c.n_p;  // a plaintext may also carry its P rows
    if (b_limbs < level || b_limbs > b_max) return set_error(CKKS_EINVAL, "second operand's limb count out of range");
    if (op == Ew::HAdd && c.windowed && b_limbs != level)
        return set_error(CKKS_EINVAL, "a windowed context takes inputs at exactly the operation level");
    for (auto [p, nm] : {std::pair<const void*, const char*>{a, "a"}, {b, "b"}, {out, "out"}})
        if (int e = check_ptr(p, nm)) return e;
    const size_t n = c.n;
    const size_t b_res = (op == Ew::HAdd ? 2 : 1) * (size_t)b_limbs * n;
    if ((out != a && overlap(out, 2 * (size_t)level * n, a, 2 * (size_t)level_a * n)) ||
        (out != b && overlap(out, 2 * (size_t)level * n, b, b_res)))
        return set_error(CKKS_EINVAL, "out partially overlaps an input");
    if ((out == a && level_a != level) || (out == b && (op != Ew::HAdd || b_limbs != level)))
        return set_error(CKKS_EINVAL, "in-place operation needs the input at the operation level");
    return launch_elementwise(c, op, a, level_a, b, b_limbs, level, out, as_stream(stream));
}

int ckks_hadd(const ckks_ctx* ctx, const uint32_t* ct_a, int level_a, const uint32_t* ct_b, int level_b, int level,
              uint32_t* out, void* stream)
{
    return elementwise(ctx, Ew::HAdd, ct_a, level_a, ct_b, level_b, level, out, stream);
}

int ckks_padd(const ckks_ctx* ctx, const uint32_t* ct, int level_in, const uint32_t* pt, int pt_limbs, int level,
              uint32_t* out, void* stream)
{
    return elementwise(ctx, Ew::PAdd, ct, level_in, pt, pt_limbs, level, out, stream);
}

int ckks_pmult(const ckks_ctx* ctx, const uint32_t* ct, int level_in, const uint32_t* pt, int pt_limbs, int level,
               uint32_t* out, void* stream)
{
    return elementwise(ctx, Ew::PMult, ct, level_in, pt, pt_limbs, level, out, stream);
}

int ckks_hconj(const ckks_ctx* ctx, const uint32_t* ct, int level_in, int level, const uint32_t* ck, uint32_t* out,
               void* ws, size_t ws_bytes, void* stream)
{
    if (int e = check_ctx(ctx)) return e;
    const Ctx& c = *ctx->impl;
    if (int e = check_level(c, level, 1)) return e;
    if (int e = check_in(c, level_in, level)) return e;
    for (auto [p, nm] : {std::pair<const void*, const char*>{ct, "ct"}, {ck, "ck"}, {out, "out"}})
        if (int e = check_ptr(p, nm)) return e;
    const size_t n = c.n;
    if (overlap(out, 2 * level * n, ct, 2 * level_in * n)) return set_error(CKKS_EINVAL, "out overlaps the input");
    if (int e = check_ws(ws, ws_bytes, keyswitch_ws_bytes(c, level))) return e;
    KsIn in;
    in.b0 = ct;
    in.a0 = ct + (size_t)level_in * n;
    in.galois = (uint32_t)(2 * n - 1);  // X -> X^(2N-1): complex conjugation of the slots
    return launch_keyswitch(c, Own::Gather, Extra::HRot, in, level, ck, out, out + (size_t)level * n, ws,
                            as_stream(stream));
}

int ckks_rescale_rational(const ckks_ctx* ctx, const uint32_t* ct, int n_in, const int32_t* in_ids, int n_out,
                          const int32_t* out_ids, uint32_t* out, void* ws, size_t ws_bytes, void* stream)
{
    if (int e = check_ctx(ctx)) return e;
    const Ctx& c = *ctx->impl;
    if (n_in < 1 || n_out < 1 || n_in > MAX_PRIMES || n_out > MAX_PRIMES || !in_ids || !out_ids)
        return set_error(CKKS_EINVAL, "bad limb counts or prime ids");
    for (int i = 0; i < n_in; i++) {
        if (in_ids[i] < 0 || in_ids[i] >= c.n_primes) return set_error(CKKS_EINVAL, "prime id out of range");
        for (int k = 0; k < i; k++)
            if (in_ids[k] == in_ids[i]) return set_error(CKKS_EINVAL, "input primes must be distinct");
    }
    for (int i = 0; i < n_out; i++) {
        if (out_ids[i] < 0 || out_ids[i] >= c.n_primes) return set_error(CKKS_EINVAL, "prime id out of range");
        for (int k = 0; k < i; k++)
            if (out_ids[k] == out_ids[i]) return set_error(CKKS_EINVAL, "output primes must be distinct");
    }
    for (auto [p, nm] : {std::pair<const void*, const char*>{ct, "ct"}, {out, "out"}})
        if (int e = check_ptr(p, nm)) return e;
    const size_t N = c.n;
    if (overlap(out, 2 * (size_t)n_out * N, ct, 2 * (size_t)n_in * N)) return set_error(CKKS_EINVAL, "out overlaps ct");
    if (int e = check_ws(ws, ws_bytes, rescale_rational_ws_bytes(c, n_in, n_out))) return e;
    if (overlap(ws, ws_bytes / 4, ct, 2 * (size_t)n_in * N) || overlap(ws, ws_bytes / 4, out, 2 * (size_t)n_out * N))
        return set_error(CKKS_EINVAL, "workspace overlaps an operand");
    return launch_rescale_rational(c, ct, n_in, in_ids, n_out, out_ids, out, ws, as_stream(stream));
}

int ckks_rescale(const ckks_ctx* ctx, const uint32_t* ct, int level, uint32_t* out, void* ws, size_t ws_bytes,
                 void* stream)
{
    if (int e = check_ctx(ctx)) return e;
    const Ctx& c = *ctx->impl;
    if (int e = check_prefix(c, "single rescaling")) return e;
    if (int e = check_level(c, level, 2)) return e;
    if (int e = check_ptr(ct, "ct")) return e;
    if (int e = check_ptr(out, "out")) return e;
    const size_t n = c.n;
    if (overlap(out, 2 * (level - 1) * n, ct, 2 * level * n)) return set_error(CKKS_EINVAL, "out overlaps the input");
    if (int e = check_ws(ws, ws_bytes, rescale_ws_bytes(c))) return e;
    return launch_rescale(c, ct, level, out, ws, as_stream(stream));
}

// ---- ciphertexts with metadata -------------------------------------------

// factor a rescaling from `level` multiplies the scale by: 1 / q_{level-1},
// or Q_A / Q_D between a window and the window below (D dropped, A added)
static double rescale_factor(const Ctx& c, int level)
{
    if (!c.windowed) return 1.0 / (double)c.mod[level - 1];
    const int below = c.rr_below[level], b0 = c.wbase[level], b1 = c.wbase[below];
    double f = 1.0;
    for (int i = b0; i < b0 + level; i++)
        if (i < b1 || i >= b1 + below) f /= (double)c.mod[i];
    for (int i = b1; i < b1 + below; i++)
        if (i < b0 || i >= b0 + level) f *= (double)c.mod[i];
    return f;
}

static int check_cts(const ckks_ct* a, const ckks_ct* b, const ckks_ct* out)
{
    if (!a || !b || !out) return set_error(CKKS_EINVAL, "null ciphertext");
    return 0;
}

int ckks_ct_hmult(const ckks_ctx* ctx, const ckks_ct* a, const ckks_ct* b, const uint32_t* rlk, int level,
                  ckks_ct* out, void* ws, size_t ws_bytes, void* stream)
{
    if (int e = check_cts(a, b, out)) return e;
    const double sc = a->scale * b->scale;
    if (int e = ckks_hmult(ctx, a->data, a->level, b->data, b->level, rlk, level, out->data, ws, ws_bytes, stream))
        return e;
    out->level = level;
    out->scale = sc;
    return CKKS_OK;
}

int ckks_ct_hmult_rescale(const ckks_ctx* ctx, const ckks_ct* a, const ckks_ct* b, const uint32_t* rlk, int level,
                          ckks_ct* out, void* ws, size_t ws_bytes, void* stream)
{
    if (int e = check_cts(a, b, out)) return e;
    const double sc = a->scale * b->scale;
    if (int e = ckks_hmult_rescale(ctx, a->data, a->level, b->data, b->level, rlk, level, out->data, ws, ws_bytes,
                                   stream))
        return e;
    const Ctx& c = *ctx->impl;
    out->level = c.rs_out(level);
    out->scale = sc * rescale_factor(c, level);
    return CKKS_OK;
}

int ckks_ct_rescale(const ckks_ctx* ctx, const ckks_ct* in, ckks_ct* out, void* ws, size_t ws_bytes, void* stream)
{
    if (int e = check_cts(in, in, out)) return e;
    const int level = in->level;
    const double sc = in->scale;
    if (int e = ckks_rescale(ctx, in->data, level, out->data, ws, ws_bytes, stream)) return e;
    out->level = level - 1;
    out->scale = sc * rescale_factor(*ctx->impl, level);
    return CKKS_OK;
}

int ckks_ct_hrot(const ckks_ctx* ctx, const ckks_ct* in, int level, int k, const uint32_t* rk, ckks_ct* out, void* ws,
                 size_t ws_bytes, void* stream)
{
    if (int e = check_cts(in, in, out)) return e;
    const double sc = in->scale;
    if (int e = ckks_hrot(ctx, in->data, in->level, level, k, rk, out->data, ws, ws_bytes, stream)) return e;
    out->level = level;
    out->scale = sc;
    return CKKS_OK;
}

}  // extern "C"
