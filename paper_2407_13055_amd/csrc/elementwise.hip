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

}  // namespace

int launch_elementwise(const Ctx& c, Ew op, const uint32_t* a, int level_a, const uint32_t* b, int level_b,
                       int level, uint32_t* out, hipStream_t s)
{
    const size_t n = c.n;
    const dim3 grid((unsigned)(n / (EW_THREADS * EW_PER_THREAD)), (unsigned)level, 2);
    const size_t ah = (size_t)level_a * n, bh = (size_t)level_b * n, oh = (size_t)level * n;
    switch (op) {
    case Ew::HAdd:
        CKKS_LAUNCH((k_elementwise<Ew::HAdd>), grid, dim3(EW_THREADS), 0, s, a, ah, b, bh, out, oh, c.mods, c.qinvs,
                    c.r1, c.log_n);
        break;
    case Ew::PAdd:
        CKKS_LAUNCH((k_elementwise<Ew::PAdd>), grid, dim3(EW_THREADS), 0, s, a, ah, b, bh, out, oh, c.mods, c.qinvs,
                    c.r1, c.log_n);
        break;
    default:
        CKKS_LAUNCH((k_elementwise<Ew::PMult>), grid, dim3(EW_THREADS), 0, s, a, ah, b, bh, out, oh, c.mods,
                    c.qinvs, c.r1, c.log_n);
    }
    return check_hip(hipGetLastError(), "element-wise launch");
}

}  // namespace ckks
