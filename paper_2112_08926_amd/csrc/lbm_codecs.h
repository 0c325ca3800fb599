// lbm_codecs.h -- conversion between FP32 (or FP64) arithmetic values and the
// DDF storage formats of Sec. 3 / Table 2 of the paper, for gfx950.
//
// Decoders are branch-free bit manipulation (one leading-bit count for the
// posits), written on the sign-extended 16-bit code that a sign-extending
// load gives, so that the sign is already at bit 31.  FP16 and FP16S use the
// hardware f32<->f16 conversions (round to nearest even).  FP16C encodes
// arithmetically (fp16c_encode).  The posits encode through a small table:
// inside one FP32 binade E the codes of these formats are either evenly
// spaced (code = first code + rounded mantissa, the carry running into the
// next binade) or absent (one threshold between the two neighbouring codes),
// so
//     code = sign | base[E] + min((mantissa + bias[E]) >> shift[E], cap[E])
// rounds every float to the nearest code with ties away from zero, and
// saturates above the largest code.  All binades below a format's window
// round to the same code (zero), all above it to the largest code, so the
// table holds only the window's 64 binades per sign, the exponent clamped
// into it; base carries the sign and bias cancels the sign and exponent bits,
// so the mantissa need not be masked out (see table_encode).  It is built on
// the host from the decoders below (lbm_enc_table.h).
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

// Small integer helpers (one instruction each on the device).
__host__ __device__ __forceinline__ uint32_t umin(uint32_t a, uint32_t b) { return a < b ? a : b; }
__host__ __device__ __forceinline__ uint32_t umax(uint32_t a, uint32_t b) { return a > b ? a : b; }
__host__ __device__ __forceinline__ uint32_t ubfe(uint32_t v, uint32_t off, uint32_t width) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_ubfe(v, off, width);
#else
    return (v >> off) & ((1u << width) - 1u);
#endif
}

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
// half up.  On the device both are computed and one selected (no branch);
// the half-up rounding is one v_cvt_rpi_i32_f32 (round to nearest, ties
// towards +infinity).  The host rounds y + 0.5 down, which is exact in
// float except just below 0.5, where y + 0.5 would round to 1: those round
// to 0.  Checked against the oracle's nearest-code encoder on all 2^32
// floats (device) and on every code boundary (host).
__host__ __device__ __forceinline__ uint16_t fp16c_encode(float x) {
    const uint32_t b = f2u(x);
    const uint32_t a = b & 0x7FFFFFFFu;
    uint32_t code;
#if defined(__HIP_DEVICE_COMPILE__)
    const uint32_t cn = umin((a - (112u << 23) + 0x800u) >> 12, 0x7FFFu);
    int32_t cd;
    asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(cd) : "v"(u2f(a) * 0x1p25f));
    code = a >= (113u << 23) ? cn : (uint32_t)cd;
#else
    if (a >= (113u << 23)) {
        code = (a - (112u << 23) + 0x800u) >> 12;
        code = code < 0x7FFFu ? code : 0x7FFFu;
    } else {
        const float y = u2f(a) * 0x1p25f;
        code = y < 0.5f ? 0u : (uint32_t)(y + 0.5f);
    }
#endif
    return (uint16_t)(((b >> 16) & 0x8000u) | code);
}

// ---------------------------------------------------------------- posits
// Sign-magnitude posits (Sec. 3.2.3): the 15 magnitude bits are placed at the
// top of a 32-bit word t; the regime is the run of equal leading bits, k long,
// with r = k - 1 for a run of ones and -k for zeros; the terminating bit is
// skipped, ES exponent bits and the fraction follow.  P16_0S / P16_1S
// additionally carry the range shift x*2^7, undone here by the exponent bias
// 127 - 7.  cs: the code sign-extended to 32 bits.
//
// On the device each decoder is one fixed instruction sequence: the run
// length is one v_ffbh_i32 (leading bits equal to bit 31; -1 for t = 0, whose
// result the zero select discards), r + 120 one v_xad_u32 ((-k ^ s) + 120),
// the fraction one v_bfe_u32.  The zero test is issued early, so that the
// select that reads its mask comes well after the compare that writes it.
template <int ES>
__host__ __device__ __forceinline__ float posit_s_decode_sext(int32_t cs) {
#if defined(__HIP_DEVICE_COMPILE__)
    uint32_t out, t, k, s, r, sh;
    if constexpr (ES == 0)
        asm("v_lshlrev_b32 %1, 17, %6\n\t"
            "v_cmp_ne_u32 vcc, 0, %1\n\t"
            "v_ffbh_i32 %2, %1\n\t"
            "v_ashrrev_i32 %3, 31, %1\n\t"
            "v_sub_u32 %4, 0, %2\n\t"
            "v_xad_u32 %4, %4, %3, %8\n\t"
            "v_lshlrev_b32 %5, %2, %1\n\t"
            "v_bfe_u32 %5, %5, 8, 23\n\t"
            "v_lshl_or_b32 %4, %4, 23, %5\n\t"
            "v_cndmask_b32 %4, 0, %4, vcc\n\t"
            "v_and_or_b32 %0, %6, %7, %4"
            : "=v"(out), "=&v"(t), "=&v"(k), "=&v"(s), "=&v"(r), "=&v"(sh)
            : "v"(cs), "s"(0x80000000u), "s"(120u)
            : "vcc");
    else                                                  // exponent bit on bit 23: r + 120 at 24, 120 = 2 * 60
        asm("v_lshlrev_b32 %1, 17, %6\n\t"
            "v_cmp_ne_u32 vcc, 0, %1\n\t"
            "v_ffbh_i32 %2, %1\n\t"
            "v_ashrrev_i32 %3, 31, %1\n\t"
            "v_sub_u32 %4, 0, %2\n\t"
            "v_xad_u32 %4, %4, %3, %8\n\t"
            "v_lshlrev_b32 %5, %2, %1\n\t"
            "v_bfe_u32 %5, %5, 7, 24\n\t"
            "v_lshl_or_b32 %4, %4, 24, %5\n\t"
            "v_cndmask_b32 %4, 0, %4, vcc\n\t"
            "v_and_or_b32 %0, %6, %7, %4"
            : "=v"(out), "=&v"(t), "=&v"(k), "=&v"(s), "=&v"(r), "=&v"(sh)
            : "v"(cs), "s"(0x80000000u), "s"(60u)
            : "vcc");
    return u2f(out);
#else
    const uint32_t t = (uint32_t)cs << 17;               // magnitude at bits 31..17, sign bits dropped
    const uint32_t s = (uint32_t)((int32_t)t >> 31);     // all ones for a run of ones
    const int k = __builtin_clz((t ^ s) | 1u);           // run length (t != 0)
    const int r = -k ^ (int)s;                           // k - 1 for ones, -k for zeros
    const uint32_t sh = t << k;                          // the terminator at bit 31
    uint32_t bits;
    if (ES == 0)
        bits = ((uint32_t)(r + 120) << 23) | ((sh >> 8) & 0x7FFFFFu);
    else
        bits = ((uint32_t)(r + 60) << 24) | ((sh >> 7) & 0xFFFFFFu);
    bits = t ? bits : 0u;
    return u2f(bits | ((uint32_t)cs & 0x80000000u));
#endif
}
template <int ES>
__host__ __device__ __forceinline__ float posit_s_decode(uint32_t c) {
    return posit_s_decode_sext<ES>((int32_t)(int16_t)(uint16_t)c);
}

// The same for codes whose regime is a run of zeros (bit 14 of the code
// clear, values below 2^-7 in magnitude): there the value is linear in the
// magnitude m.  With es = 0, m = 2^(14-k) (1 + f / 2^(14-k)) for a run of k
// zeros and the value 2^(-k-7) (1 + f / 2^(14-k)) = m 2^-21; with es = 1 the
// float of m has exponent field 141 - k and e at the top of its mantissa, so
// its bits shifted left by one carry (2 (141 - k) + e) in the exponent field,
// from which 162 is taken to reach 120 - 2k + e.  Code 0 (0.0) gives garbage
// that the minimum with the float's own bits (0) removes, as for P16_2C.
template <int ES>
__host__ __device__ __forceinline__ float posit_s_decode_zeros_run(int32_t cs) {
    const uint32_t mag = (uint32_t)cs & 0x3FFFu;
    const uint32_t b = f2u((float)mag);                    // exact: mag < 2^14
    const uint32_t bits = ES == 0 ? umin(b - (21u << 23), b) : umin((b << 1) - (162u << 23), b);
    return u2f(bits | ((uint32_t)cs & 0x80000000u));
}

// P16_0S encoder for |x| < 2^-7, where its codes are the fixed-point values
// m 2^-21 (the run-of-zeros codes above; the next code, 0x4000, is 2^-7
// itself and also m 2^-21): the nearest code, ties away from zero, is |x|
// 2^21 rounded half up, one v_cvt_rpi_i32_f32 on the device (as in the
// FP16C encoder's denormal range), with the sign of x.  Equal to the table
// encoder there (checked on the host for every such float, and on the
// device as part of the exhaustive encode test).
constexpr float kP160sFixedBound = 0x1p-7f;
__host__ __device__ __forceinline__ uint16_t p160s_encode_fixed(float x) {
    const uint32_t b = f2u(x);
    const float y = u2f(b & 0x7FFFFFFFu) * 0x1p21f;       // exact: a power of two
#if defined(__HIP_DEVICE_COMPILE__)
    int32_t m;
    asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(m) : "v"(y));
#else
    const int32_t m = y < 0.5f ? 0 : (int32_t)(y + 0.5f);  // y + 0.5 exact for y in [0.5, 2^14]
#endif
    return (uint16_t)(((b >> 16) & 0x8000u) | (uint32_t)m);
}

// Asymmetric P16_2C: r leading zeros close with a one (no regime sign), then
// 2 exponent bits and 12 - r mantissa bits; value 2^(-3-4r+e)(1 + m/2^(12-r)).
// The 15-bit magnitude converted to float does the regime count: its leading
// one is at bit 14 - r, so the float's exponent field is 141 - r and its
// mantissa holds e at the top, then m.  Shifting the float's bits left by 2
// multiplies the exponent field by 4 and moves e into its low bits, leaving
// m in place of the mantissa: (4 (141 - r) + e) mod 512 at bits 31..23, from
// which 440 is taken to reach 124 - 4r + e (68 .. 127 for every code, so the
// modular arithmetic ends in range).  Code 0 converts to 0.0, whose shifted
// bits give garbage: the minimum with the float's own bits (0 there, and
// above every result for any other code, which converts to 1.0 or more)
// maps it to 0.  Five instructions with the sign.
__host__ __device__ __forceinline__ float p162c_decode_sext(int32_t cs) {
    const uint32_t mag = (uint32_t)cs & 0x7FFFu;
    const uint32_t b = f2u((float)mag);                    // exact: mag < 2^15
    const uint32_t bits = umin((b << 2) - (440u << 23), b);
    return u2f(bits | ((uint32_t)cs & 0x80000000u));
}
__host__ __device__ __forceinline__ float p162c_decode(uint32_t c) {
    return p162c_decode_sext((int32_t)(int16_t)(uint16_t)c);
}

// ---------------------------------------------------------------- IEEE FP16
__host__ __device__ __forceinline__ float half_decode(uint32_t c) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)c);
}
__host__ __device__ __forceinline__ uint16_t half_encode(float x) {
    return __builtin_bit_cast(uint16_t, (_Float16)x);
}

// First FP32 exponent field of a posit format's encoder window: two binades
// below its smallest code (the lower one rounds to zero, the upper one to
// the smallest code); the window's last binade lies above the largest code.
__host__ __device__ constexpr uint32_t enc_window_lo(int fmt) {
    return fmt == S_P16_0S ? 104u : fmt == S_P16_1S ? 90u : fmt == S_P16_2C ? 66u : 0u;
}

// Software encoder through the windowed per-binade table (kEncEntries
// entries, kEncWindow per sign) of the format whose window starts at lo.
// On the device the table is in LDS (every caller stages it there) and the
// entry's address is one fixed sequence: the exponent field (v_bfe_u32),
// clamped into the window (v_med3_u32), plus the sign's half (two
// v_lshl_add_u32); then one 16-byte LDS read.
__host__ __device__ __forceinline__ uint16_t table_encode(float x, const EncEntry* tab, uint32_t lo) {
    const uint32_t b = f2u(x);
#if defined(__HIP_DEVICE_COMPILE__)
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    typedef const __attribute__((address_space(3))) u32x4* LdsEntry;
    // LDS address of the entry of exponent 0 of the positive half (the
    // clamped exponent is added to it, scaled by the entry size)
    const uint32_t t0 = (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) EncEntry*)tab - lo * 16u;
    uint32_t addr, e, sg;
    asm("v_bfe_u32 %1, %3, 23, 8\n\t"
        "v_med3_u32 %1, %1, %5, %6\n\t"
        "v_lshrrev_b32 %2, 31, %3\n\t"
        "v_lshl_add_u32 %0, %2, %7, %4\n\t"
        "v_lshl_add_u32 %0, %1, 4, %0"
        : "=&v"(addr), "=&v"(e), "=&v"(sg)
        : "v"(b), "s"(t0), "s"(lo), "v"(lo + (kEncWindow - 1)), "i"(__builtin_ctz(kEncWindow * 16)));
    const u32x4 ent = *(LdsEntry)(uintptr_t)addr;          // base, cap, bias, shift
    uint32_t j = (b + ent.z) >> ent.w;
    j = j < ent.y ? j : ent.y;
    return (uint16_t)(ent.x + j);
#else
    const uint32_t E = umin(umax(ubfe(b, 23, 8), lo), lo + (kEncWindow - 1));
    const EncEntry e = tab[((b >> 31) * kEncWindow) + (E - lo)];
    uint32_t j = (b + e.bias) >> e.shift;
    j = j < e.cap ? j : e.cap;
    return (uint16_t)(e.base + j);
#endif
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

// Formats with an arithmetic encoder for a range of small values (used by
// wavefronts whose values all lie there; the others take the table).  Its
// store() takes the values the step stores, which for these formats are the
// physical ones (raw units 2^-0).
template <int F> struct FixedRange { static constexpr bool value = false; };
template <> struct FixedRange<S_P16_0S> {
    static constexpr bool value = true;
    static constexpr float kBound = kP160sFixedBound;   // |x| < kBound
    __device__ __forceinline__ static uint16_t store(float x) { return p160s_encode_fixed(x); }
};

// Formats with a cheaper decoder for the codes whose regime is a run of
// zeros (bit 14 clear): the sign-magnitude posits P16_0S and P16_1S.
template <int F> struct ZerosRun { static constexpr bool value = false; };
template <> struct ZerosRun<S_P16_0S> {
    static constexpr bool value = true;
    template <class A> __device__ __forceinline__ static A load(uint16_t v) {
        return posit_s_decode_zeros_run<0>((int16_t)v);
    }
};
template <> struct ZerosRun<S_P16_1S> {
    static constexpr bool value = true;
    template <class A> __device__ __forceinline__ static A load(uint16_t v) {
        return posit_s_decode_zeros_run<1>((int16_t)v);
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
    template <class A> __device__ __forceinline__ static A load(T v) { return posit_s_decode_sext<0>((int16_t)v); }
    template <class A> __device__ __forceinline__ static T store(A v, const EncEntry* t) {
        return table_encode(v, t, enc_window_lo(S_P16_0S));
    }
};
template <> struct Codec<S_P16_1S> : RawCodec<S_P16_1S> {
    using T = uint16_t;
    static constexpr int kRawExp = 0;
    static constexpr bool kTable = true;
    template <class A> __device__ __forceinline__ static A load(T v) { return posit_s_decode_sext<1>((int16_t)v); }
    template <class A> __device__ __forceinline__ static T store(A v, const EncEntry* t) {
        return table_encode(v, t, enc_window_lo(S_P16_1S));
    }
};
template <> struct Codec<S_P16_2C> : RawCodec<S_P16_2C> {
    using T = uint16_t;
    static constexpr int kRawExp = 0;
    static constexpr bool kTable = true;
    template <class A> __device__ __forceinline__ static A load(T v) { return p162c_decode_sext((int16_t)v); }
    template <class A> __device__ __forceinline__ static T store(A v, const EncEntry* t) {
        return table_encode(v, t, enc_window_lo(S_P16_2C));
    }
};

}  // namespace lbm
