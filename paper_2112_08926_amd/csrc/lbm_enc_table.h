// lbm_enc_table.h -- host construction of the software encoder tables of
// FP16C and the posit formats (see lbm_codecs.h for how they are used).
#pragma once

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "lbm_codecs.h"

namespace lbm {

// For FP16C and the posits: per FP32 binade E (exponent field of |x|), the
// parameters of code = base + min((mantissa + bias) >> shift, cap); built
// from the decoders of lbm_codecs.h so that encode(x) is the nearest code
// (ties away from zero), saturating at the largest magnitude code.
inline bool build_encoder_table(int fmt, EncEntry out[256], std::string* why) {
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
                if (mid < lo) e.bias = 1u << 23;
                else if (mid >= hi) e.bias = 0;
                else {
                    const double mthr = (mid / lo - 1.0) * 8388608.0;
                    if (mthr != std::floor(mthr)) { *why = "midpoint not a float"; return false; }
                    e.bias = (1u << 23) - (uint32_t)mthr;
                }
            }
        }
        out[E] = e;
    }
    return true;
}

}  // namespace lbm
