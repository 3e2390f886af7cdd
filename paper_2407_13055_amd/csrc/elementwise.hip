// Element-wise mechanisms of Sec. 2.1 on evaluation-domain ciphertexts:
// HAdd (component-wise sum), PAdd (plaintext added to the b half), PMult
// (both halves times a plaintext, slot-wise).  HBM-bound: each thread moves
// 16-byte runs (4 residues) of one limb; grid = (N / 1024, level, 2 halves).
#include <hip/hip_runtime.h>

#include "internal.h"
#include "modarith.h"

namespace ckks {

namespace {

constexpr int EW_THREADS = 256;
constexpr int EW_PER_THREAD = 4;

template <Ew OP>
__global__ void __launch_bounds__(EW_THREADS) k_elementwise(const uint32_t* a, size_t a_half, const uint32_t* b,
                                                           size_t b_half, uint32_t* out, size_t o_half,
                                                           const uint32_t* mods, const uint32_t* qinvs,
                                                           const uint2* r1, int log_n)
{
    const int limb = blockIdx.y, half = blockIdx.z;
    const size_t j = ((size_t)blockIdx.x * EW_THREADS + threadIdx.x) * EW_PER_THREAD;  // exact grid
    const size_t off = ((size_t)limb << log_n) + j;
    const uint32_t q = mods[limb];
    const uint4 x = *reinterpret_cast<const uint4*>(a + half * a_half + off);
    uint4 r;
    if constexpr (OP == Ew::HAdd) {
        const uint4 y = *reinterpret_cast<const uint4*>(b + half * b_half + off);
        r = make_uint4(add_mod(x.x, y.x, q), add_mod(x.y, y.y, q), add_mod(x.z, y.z, q), add_mod(x.w, y.w, q));
    } else if constexpr (OP == Ew::PAdd) {
        if (half == 0) {
            const uint4 y = *reinterpret_cast<const uint4*>(b + off);
            r = make_uint4(add_mod(x.x, y.x, q), add_mod(x.y, y.y, q), add_mod(x.z, y.z, q), add_mod(x.w, y.w, q));
        } else {
            r = x;
        }
    } else {  // PMult: mont gives x m 2^-32, the twisted constant R restores x m (canonical)
        const uint4 y = *reinterpret_cast<const uint4*>(b + off);
        const uint32_t qinv = qinvs[limb];
        const uint2 c = r1[limb];
        r = make_uint4(mulc(mont(x.x, y.x, q, qinv), c, q), mulc(mont(x.y, y.y, q, qinv), c, q),
                       mulc(mont(x.z, y.z, q, qinv), c, q), mulc(mont(x.w, y.w, q, qinv), c, q));
    }
    *reinterpret_cast<uint4*>(out + half * o_half + off) = r;
}

__global__ void __launch_bounds__(EW_THREADS) k_lincomb(LincombArgs L, const uint32_t* x, size_t x_half,
                                                       const uint32_t* y, size_t y_half, uint32_t* out,
                                                       size_t o_half, int log_n)
{
    const int limb = blockIdx.y, half = blockIdx.z;
    const size_t j = ((size_t)blockIdx.x * EW_THREADS + threadIdx.x) * EW_PER_THREAD;
    const uint32_t q = L.q[limb];
    const int xr = L.xrow[limb];
    uint32_t r[4] = {0, 0, 0, 0};
    if (xr >= 0) {
        const uint4 v = *reinterpret_cast<const uint4*>(x + half * x_half + ((size_t)xr << log_n) + j);
        const uint2 a = L.a[limb];
        r[0] = mulc(v.x, a, q), r[1] = mulc(v.y, a, q), r[2] = mulc(v.z, a, q), r[3] = mulc(v.w, a, q);
    }
    if (y) {
        const uint4 v = *reinterpret_cast<const uint4*>(y + half * y_half + ((size_t)limb << log_n) + j);
        const uint2 b = L.b[limb];
        r[0] = add_mod(r[0], mulc(v.x, b, q), q), r[1] = add_mod(r[1], mulc(v.y, b, q), q);
        r[2] = add_mod(r[2], mulc(v.z, b, q), q), r[3] = add_mod(r[3], mulc(v.w, b, q), q);
    }
    *reinterpret_cast<uint4*>(out + half * o_half + ((size_t)limb << log_n) + j) = make_uint4(r[0], r[1], r[2], r[3]);
}

}  // namespace

int launch_lincomb(const Ctx& c, const LincombArgs& L, const uint32_t* x, size_t x_half, const uint32_t* y,
                   size_t y_half, uint32_t* out, size_t o_half, hipStream_t s)
{
    const dim3 grid((unsigned)(c.n / (EW_THREADS * EW_PER_THREAD)), (unsigned)L.n, 2);
    CKKS_LAUNCH(k_lincomb, grid, dim3(EW_THREADS), 0, s, L, x, x_half, y, y_half, out, o_half, c.log_n);
    return check_hip(hipGetLastError(), "linear-combination launch");
}

int launch_elementwise(const Ctx& c, Ew op, const uint32_t* a, int level_a, const uint32_t* b, int level_b,
                       int level, uint32_t* out, hipStream_t s)
{
    const size_t n = c.n;
    const dim3 grid((unsigned)(n / (EW_THREADS * EW_PER_THREAD)), (unsigned)level, 2);
    const size_t ah = (size_t)level_a * n, bh = (size_t)level_b * n, oh = (size_t)level * n;
    const int wb = c.wbase[level];  // limb i has prime id wb + i
    const uint32_t* mods = c.mods + wb;
    const uint32_t* qinvs = c.qinvs + wb;
    const uint2* r1 = c.r1 + wb;
    switch (op) {
    case Ew::HAdd:
        CKKS_LAUNCH((k_elementwise<Ew::HAdd>), grid, dim3(EW_THREADS), 0, s, a, ah, b, bh, out, oh, mods, qinvs, r1,
                    c.log_n);
        break;
    case Ew::PAdd:
        CKKS_LAUNCH((k_elementwise<Ew::PAdd>), grid, dim3(EW_THREADS), 0, s, a, ah, b, bh, out, oh, mods, qinvs, r1,
                    c.log_n);
        break;
    default:
        CKKS_LAUNCH((k_elementwise<Ew::PMult>), grid, dim3(EW_THREADS), 0, s, a, ah, b, bh, out, oh, mods, qinvs,
                    r1, c.log_n);
    }
    return check_hip(hipGetLastError(), "element-wise launch");
}

}  // namespace ckks
