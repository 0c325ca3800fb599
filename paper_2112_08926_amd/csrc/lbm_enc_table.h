// lbm_enc_table.h -- host construction of the software encoder tables of
// FP16C and the posit formats (see lbm_codecs.h for how they are used).
#pragma once

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "lbm_codecs.h"

namespace lbm {

// For the posits: per FP32 binade E (exponent field of |x|), the parameters
// of code = base + min((mantissa + bias) >> shift, cap); built from the
// decoders of lbm_codecs.h so that encode(x) is the nearest code (ties away
// from zero), saturating at the largest magnitude code.  The device table
// keeps the binades lo .. lo + kEncWindow - 1 of the format's window (the
// encoder clamps the exponent into it), which is only exact if every binade
// below the window encodes like its first one and every binade above like
// its last one, each to a single code (cap 0): checked here.  Entry s *
// kEncWindow + (E - lo) serves sign s in binade E: its base carries the sign
// bit (0x8000) and its bias has the 9 sign and exponent bits (s * 256 + E)
// << 23 subtracted (mod 2^32), so that table_encode adds it to the whole FP32
// word instead of the masked mantissa.
inline bool build_encoder_table(int fmt, EncEntry out[kEncEntries], std::string* why) {
    EncEntry full[256];
    const int maxc = 0x7FFF;
    std::vector<double> v(maxc + 1);
    for (int c = 0; c <= maxc; c++) v[c] = (double)decode16(fmt, (uint32_t)c);
    for (int c = 1; c <= maxc; c++)
        if (!(v[c] > v[c - 1])) { *why = "decoder not monotone"; return false; }
    for (int E = 0; E < 256; E++) {
        EncEntry e{0, 0, 0, 23};
        if (E == 0) {                 // FP32 zero/denormals: below every positive code
            e = {0, 0, 0, 23};
        } else if (E == 255) {        // Inf/NaN saturate
            e = {(uint32_t)maxc, 0, 0, 23};
        } else {
            const double lo = std::ldexp(1.0, E - 127), hi = 2.0 * lo;
            const int cf = (int)(std::lower_bound(v.begin(), v.end(), lo) - v.begin());
            if (cf > maxc) {
                e = {(uint32_t)maxc, 0, 0, 23};
            } else if (v[cf] < hi) {
                // populated binade: evenly spaced codes starting at lo
                if (v[cf] != lo) { *why = "binade does not start at a power of two"; return false; }
                int cnt = 0;
                while (cf + cnt <= maxc && v[cf + cnt] < hi) cnt++;
                int nm = 0;
                while ((1 << nm) < cnt) nm++;
                if ((1 << nm) != cnt || nm > 23) { *why = "binade count not a power of two"; return false; }
                for (int j = 0; j < cnt; j++)
                    if (v[cf + j] != lo * (1.0 + std::ldexp((double)j, -nm))) { *why = "uneven binade"; return false; }
                const uint32_t shift = 23 - nm;
                e.base = (uint32_t)cf;
                e.shift = shift;
                e.bias = shift ? (1u << (shift - 1)) : 0u;
                const bool next_is_hi = (cf + cnt <= maxc) && v[cf + cnt] == hi;
                e.cap = (uint32_t)(next_is_hi ? cnt : cnt - 1);
            } else {
                // empty binade: the nearest code is v[cf-1] or v[cf]
                const int cp = cf - 1;
                const double mid = 0.5 * (v[cp] + v[cf]);
                e.base = (uint32_t)cp;
                e.cap = 1;
                e.shift = 23;
                if (mid < lo) e = {(uint32_t)cf, 0, 0, 23};          // the whole binade rounds up
                else if (mid >= hi) e = {(uint32_t)cp, 0, 0, 23};    // ... or down
                else {
                    const double mthr = (mid / lo - 1.0) * 8388608.0;
                    if (mthr != std::floor(mthr)) { *why = "midpoint not a float"; return false; }
                    e.bias = (1u << 23) - (uint32_t)mthr;
                }
            }
        }
        full[E] = e;
    }
    const uint32_t lo = enc_window_lo(fmt), hi = lo + kEncWindow - 1;
    if (lo == 0 || full[lo].cap != 0 || full[hi].cap != 0) {
        *why = "window edges are not single-code binades";
        return false;
    }
    for (uint32_t E = 0; E < 256; E++)
        if ((E < lo && full[E].base != full[lo].base) || (E > hi && full[E].base != full[hi].base) ||
            ((E < lo || E > hi) && full[E].cap != 0)) {
            *why = "a binade outside the window encodes unlike the window's edge";
            return false;
        }
    for (uint32_t sgn = 0; sgn < 2; sgn++)
        for (uint32_t w = 0; w < (uint32_t)kEncWindow; w++) {
            const EncEntry& e = full[lo + w];
            const uint32_t idx = sgn * 256u + lo + w;
            out[sgn * kEncWindow + w] = {e.base | (sgn << 15), e.cap, e.bias - (idx << 23), e.shift};
        }
    return true;
}

}  // namespace lbm
