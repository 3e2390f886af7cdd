// Device-side 32-bit modular arithmetic for RNS primes q < 2^31 on the
// integer VALU of gfx950 (v_mul_lo_u32 / v_mul_hi_u32 / v_mad_i64_i32).
//
// Reductions (Sec. 4.1, Alg. 2 and Table 3):
//  * mont(a, b)        a*b*2^-32 mod q for data x data products (Montgomery;
//                      the 2^-32 factors are folded into precomputed
//                      constants downstream, Sec. 5.1 Seq.2).
//  * mulc(x, W, Wt)    x*w mod q for a known constant w, stored "twisted":
//                      W = w*2^32 mod q and Wt = W*q^-1 mod 2^32, so the
//                      Montgomery quotient needs no product of x with a
//                      data-dependent value: 3 multiplies, 3 adds, output
//                      canonical in [0, q) for any 32-bit x.
//  * smr64(x, t, tinv) signed Montgomery reduction (Seiler's signed variant
//                      of Montgomery's method) of a 64-bit signed sum: the
//                      reduction Sec. 4.1 picks for base conversion.
//  All outputs are canonical [0, q) unless stated.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ckks {

// r in (-q, q) held as a wrapped uint32 -> [0, q)
__device__ __forceinline__ uint32_t fix_signed(uint32_t r, uint32_t q) { return min(r, r + q); }

__device__ __forceinline__ uint32_t add_mod(uint32_t a, uint32_t b, uint32_t q)
{
    uint32_t r = a + b;  // < 2q < 2^32
    return min(r, r - q);
}

__device__ __forceinline__ uint32_t sub_mod(uint32_t a, uint32_t b, uint32_t q) { return fix_signed(a - b, q); }

// x * w mod q, (W, Wt) = (w*2^32 mod q, W*q^-1 mod 2^32); any x < 2^32.
__device__ __forceinline__ uint32_t mulc(uint32_t x, uint32_t W, uint32_t Wt, uint32_t q)
{
    uint32_t hi = __umulhi(x, W);
    uint32_t t = __umulhi(x * Wt, q);
    return fix_signed(hi - t, q);
}

__device__ __forceinline__ uint32_t mulc(uint32_t x, uint2 w, uint32_t q) { return mulc(x, w.x, w.y, q); }

// a*b*2^-32 mod q for a*b < q*2^32 (e.g. both canonical).
__device__ __forceinline__ uint32_t mont(uint32_t a, uint32_t b, uint32_t q, uint32_t qinv)
{
    uint32_t lo = a * b;
    uint32_t hi = __umulhi(a, b);
    uint32_t t = __umulhi(lo * qinv, q);
    return fix_signed(hi - t, q);
}

// Shoup multiplication by a constant w < q with ws = floor(w 2^32 / q):
// x*w - floor(x ws / 2^32) q lies in [0, 2q) for any 32-bit x (2 multiplies
// by known constants, one by the quotient estimate).
__device__ __forceinline__ uint32_t mul_shoup(uint32_t x, uint32_t w, uint32_t ws, uint32_t q)
{
    return x * w - __umulhi(x, ws) * q;
}

// the same product negated modulo 2^32: 2^32 - (x w mod q in [0, 2q)), or 0
__device__ __forceinline__ uint32_t mul_shoup_neg(uint32_t x, uint32_t w, uint32_t ws, uint32_t q)
{
    return __umulhi(x, ws) * q - x * w;
}

// [0, 2m) -> [0, m)
__device__ __forceinline__ uint32_t red2(uint32_t x, uint32_t m) { return min(x, x - m); }

// twisted companion of a Montgomery-form constant W
__device__ __forceinline__ uint2 twist(uint32_t W, uint32_t qinv) { return make_uint2(W, W * qinv); }

// Signed Montgomery reduction: r = x 2^-32 (mod t) with |r| < t, for odd
// t < 2^31, tinv = t^-1 mod 2^32 and |x| <= t 2^31.
// Why it works: m = x t^-1 mod 2^32, read as a signed 32-bit value, makes
// x - m t divisible by 2^32; x and m t then share their low 32 bits, so the
// exact quotient (x - m t) / 2^32 is the difference of their high halves.
// |x / 2^32| <= t/2 and |m t / 2^32| <= t/2 bound it by t.
__device__ __forceinline__ int32_t smr64(int64_t x, uint32_t t, uint32_t tinv)
{
    const int32_t m = (int32_t)((uint32_t)x * tinv);
    return (int32_t)(x >> 32) - __mulhi(m, (int32_t)t);
}

// (-t, t) -> [0, t)
__device__ __forceinline__ uint32_t canon_signed(int32_t y, uint32_t t) { return (uint32_t)(y < 0 ? y + (int32_t)t : y); }

// centred representative of v in [0, q): v if 2v < q else v - q
__device__ __forceinline__ int32_t lift(uint32_t v, uint32_t q) { return (int32_t)(v > (q >> 1) ? v - q : v); }

// reduce a centred int32 into [0, t); one conditional add when |y| < t (the
// case for lifted residues of a prime of the same size), a division otherwise
__device__ __forceinline__ uint32_t reduce_centred(int32_t y, uint32_t t)
{
    uint32_t u = y < 0 ? (uint32_t)(y + (int32_t)t) : (uint32_t)y;
    if (u >= t) {
        int32_t r = y % (int32_t)t;
        u = (uint32_t)(r < 0 ? r + (int32_t)t : r);
    }
    return u;
}

}  // namespace ckks
