// lbm_codecs.h -- conversion between FP32 (or FP64) arithmetic values and the
// DDF storage formats of Sec. 3 / Table 2 of the paper, for gfx950.
//
// Decoders are branch-free bit manipulation (one leading-zero count for the
// posits).  FP16 and FP16S use the hardware f32<->f16 conversions (round to
// nearest even).  FP16C encodes arithmetically (fp16c_encode).  The posits
// encode through a 256-entry table
// indexed by the FP32 exponent field: inside one FP32 binade the codes of
// these formats are either evenly spaced (code = first code + rounded
// mantissa, the carry running into the next binade) or absent (one threshold
// between the two neighbouring codes), so
//     code = base[E] + min((mantissa + bias[E]) >> shift[E], cap[E])
// rounds every float to the nearest code with ties away from zero, and
// saturates above the largest code.  The table is built on the host from
// the decoders below (build_encoder_table in the runtime).
//
// Every function here is __host__ __device__ so that the host can build the
// tables from exactly the device decoders.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_internal.h"

namespace lbm {

__host__ __device__ __forceinline__ uint32_t f2u(float x) { return __builtin_bit_cast(uint32_t, x); }
__host__ __device__ __forceinline__ float u2f(uint32_t u) { return __builtin_bit_cast(float, u); }

// ---------------------------------------------------------------- FP16C
// 1 sign | 4 exponent (bias 15) | 11 mantissa, no Inf/NaN.  Placing the 15
// magnitude bits at FP32 bits 26..12 gives 2^(e-127)(1 + m/2^11), or the FP32
// denormal m 2^-137 for e = 0; one multiply by 2^112 rebiases both exactly.
// From the sign-extended code (what a sign-extending 16-bit load gives):
// shifted by 12, its bits 31..27 are all the sign, so one mask keeps the sign
// at bit 31 and the magnitude at bits 26..12.
__host__ __device__ __forceinline__ float fp16c_decode_sext(int32_t cs) {
    return u2f(((uint32_t)cs << 12) & 0x87FFF000u) * 0x1p112f;
}
__host__ __device__ __forceinline__ float fp16c_decode(uint32_t c) {
    return fp16c_decode_sext((int32_t)(int16_t)(uint16_t)c);
}

// Nearest FP16C code, ties away from zero, saturating at 0x7FFF (NaN too).
// |x| >= 2^-14: the FP32 bits rebiased by 112 in the exponent, rounded at
// the 12th bit (a carry moves to the next binade by itself).  Below: the
// denormal codes are the multiples of 2^-25, so the code is |x| 2^25 rounded
// half up (exact in float except just below 0.5, where y + 0.5 would round
// to 1: those round to 0).  Checked against the exact table encoder on all
// 2^32 floats.
__host__ __device__ __forceinline__ uint16_t fp16c_encode(float x) {
    const uint32_t b = f2u(x);
    const uint32_t a = b & 0x7FFFFFFFu;
    uint32_t code;
    if (a >= (113u << 23)) {
        code = (a - (112u << 23) + 0x800u) >> 12;
        code = code < 0x7FFFu ? code : 0x7FFFu;
    } else {
        const float y = u2f(a) * 0x1p25f;
        code = y < 0.5f ? 0u : (uint32_t)(y + 0.5f);
    }
    return (uint16_t)(((b >> 16) & 0x8000u) | code);
}

// ---------------------------------------------------------------- posits
// Sign-magnitude posits (Sec. 3.2.3): the 15 magnitude bits are placed at the
// top of a 32-bit word; the regime is the run of equal leading bits.
// P16_0S / P16_1S additionally carry the range shift x*2^7, undone here by
// the exponent bias 127 - 7.
template <int ES>
__host__ __device__ __forceinline__ float posit_s_decode(uint32_t c) {
    const uint32_t mag = c & 0x7FFFu;
    const uint32_t t = mag << 17;
    const uint32_t s = (uint32_t)((int32_t)t >> 31);     // all ones for a regime of ones (r >= 0)
    const int k = __builtin_clz((t ^ s) | 1u);           // run length (mag != 0)
    const int r = (k - 1) ^ (int)~s;                     // k - 1 for ones, -k for zeros
    const uint32_t sh = t << k;                          // the terminator at bit 31
    uint32_t bits;
    if (ES == 0)
        bits = ((uint32_t)r << 23) + ((sh >> 8) & 0x7FFFFFu) + (120u << 23);
    else
        bits = ((uint32_t)r << 24) + ((sh >> 7) & 0xFFFFFFu) + (120u << 23);   // exponent bit on bit 23
    bits = mag ? bits : 0u;
    return u2f(bits | ((c & 0x8000u) << 16));
}

// Asymmetric P16_2C: r leading zeros close with a one (no regime sign), then
// 2 exponent bits and 12 - r mantissa bits; value 2^(-3-4r+e)(1 + m/2^(12-r)).
__host__ __device__ __forceinline__ float p162c_decode(uint32_t c) {
    const uint32_t mag = c & 0x7FFFu;
    const uint32_t t = mag << 17;
    const int r = __builtin_clz(t | 1u);
    const uint32_t rest = (t << r) << 1;                 // exponent bits at 31..30
    uint32_t bits = (uint32_t)((124 - 4 * r) << 23) + (rest >> 7);
    bits = mag ? bits : 0u;
    return u2f(bits | ((c & 0x8000u) << 16));
}

// ---------------------------------------------------------------- IEEE FP16
__host__ __device__ __forceinline__ float half_decode(uint32_t c) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)c);
}
__host__ __device__ __forceinline__ uint16_t half_encode(float x) {
    return __builtin_bit_cast(uint16_t, (_Float16)x);
}

// Software encoder through the per-binade table.
__host__ __device__ __forceinline__ uint16_t table_encode(float x, const EncEntry* tab) {
    const uint32_t b = f2u(x);
    const uint32_t a = b & 0x7FFFFFFFu;
    const EncEntry e = tab[a >> 23];
    uint32_t j = ((a & 0x7FFFFFu) + e.bias) >> e.shift;
    j = j < e.cap ? j : e.cap;
    return (uint16_t)(((b >> 16) & 0x8000u) | (e.base + j));
}

// Decoded value of a 16-bit code of a format (host table builder and tests).
__host__ __device__ __forceinline__ float decode16(int fmt, uint32_t c) {
    switch (fmt) {
    case S_FP16:   return half_decode(c);
    case S_FP16S:  return half_decode(c) * 0x1p-15f;
    case S_FP16C:  return fp16c_decode(c);
    case S_P16_0S: return posit_s_decode<0>(c);
    case S_P16_1S: return posit_s_decode<1>(c);
    case S_P16_2C: return p162c_decode(c);
    default:       return 0.0f;
    }
}

// ---------------------------------------------------------------- storage traits
// Codec<F>::T is the stored type; load() returns the arithmetic value, store()
// takes it.  `tab` is the encoder table in LDS (used by FP16C and posits).
// load_raw()/store_raw() work in units of 2^-kRawExp: the step kernel does
// its arithmetic in those units (every constant scaled by 2^kRawExp; scaling
// by a power of two is exact, so the result is the same), which removes the
// FP16S range shift from every load and store.
template <int F> struct Codec;

template <int F>
struct RawCodec {
    template <class A, class TT> __device__ __forceinline__ static A load_raw(TT v) {
        return Codec<F>::template load<A>(v);
    }
    template <class A> __device__ __forceinline__ static auto store_raw(A v, const EncEntry* t) {
        return Codec<F>::template store<A>(v, t);
    }
};

template <> struct Codec<S_FP64> : RawCodec<S_FP64> {
    using T = double;
    static constexpr int kRawExp = 0;
    static constexpr bool kTable = false;
    template <class A> __device__ __forceinline__ static A load(T v) { return (A)v; }
    template <class A> __device__ __forceinline__ static T store(A v, const EncEntry*) { return (T)v; }
};
template <> struct Codec<S_FP32> : RawCodec<S_FP32> {
    using T = float;
    static constexpr int kRawExp = 0;
    static constexpr bool kTable = false;
    template <class A> __device__ __forceinline__ static A load(T v) { return (A)v; }
    template <class A> __device__ __forceinline__ static T store(A v, const EncEntry*) { return (T)v; }
};
template <> struct Codec<S_FP16> : RawCodec<S_FP16> {
    using T = uint16_t;
    static constexpr int kRawExp = 0;
    static constexpr bool kTable = false;
    template <class A> __device__ __forceinline__ static A load(T v) { return half_decode(v); }
    template <class A> __device__ __forceinline__ static T store(A v, const EncEntry*) { return half_encode(v); }
};
template <> struct Codec<S_FP16S> {
    using T = uint16_t;
    static constexpr int kRawExp = 15;          // the stored FP16 value is x * 2^15
    static constexpr bool kTable = false;
    template <class A> __device__ __forceinline__ static A load(T v) { return half_decode(v) * 0x1p-15f; }
    // The 2^15 scale is an exponent add (ldexp: exact, keeps -0); a plain
    // multiply gets fused with the conversion into a multiply-add with a +0
    // addend, which would turn -0 into +0.
    template <class A> __device__ __forceinline__ static T store(A v, const EncEntry*) {
        return half_encode(__builtin_ldexpf(v, 15));
    }
    template <class A> __device__ __forceinline__ static A load_raw(T v) { return half_decode(v); }
    template <class A> __device__ __forceinline__ static T store_raw(A v, const EncEntry*) { return half_encode(v); }
};
template <> struct Codec<S_FP16C> : RawCodec<S_FP16C> {
    using T = uint16_t;
    static constexpr int kRawExp = 0;
    static constexpr bool kTable = false;            // arithmetic encoder
    template <class A> __device__ __forceinline__ static A load(T v) { return fp16c_decode_sext((int16_t)v); }
    template <class A> __device__ __forceinline__ static T store(A v, const EncEntry*) { return fp16c_encode(v); }
};
template <> struct Codec<S_P16_0S> : RawCodec<S_P16_0S> {
    using T = uint16_t;
    static constexpr int kRawExp = 0;
    static constexpr bool kTable = true;
    template <class A> __device__ __forceinline__ static A load(T v) { return posit_s_decode<0>(v); }
    template <class A> __device__ __forceinline__ static T store(A v, const EncEntry* t) { return table_encode(v, t); }
};
template <> struct Codec<S_P16_1S> : RawCodec<S_P16_1S> {
    using T = uint16_t;
    static constexpr int kRawExp = 0;
    static constexpr bool kTable = true;
    template <class A> __device__ __forceinline__ static A load(T v) { return posit_s_decode<1>(v); }
    template <class A> __device__ __forceinline__ static T store(A v, const EncEntry* t) { return table_encode(v, t); }
};
template <> struct Codec<S_P16_2C> : RawCodec<S_P16_2C> {
    using T = uint16_t;
    static constexpr int kRawExp = 0;
    static constexpr bool kTable = true;
    template <class A> __device__ __forceinline__ static A load(T v) { return p162c_decode(v); }
    template <class A> __device__ __forceinline__ static T store(A v, const EncEntry* t) { return table_encode(v, t); }
};

}  // namespace lbm
