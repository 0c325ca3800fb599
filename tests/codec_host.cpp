// Host build of the library's codec header (the same decoders and encoder
// table the kernels use), for a CPU comparison with the oracle:
//   codec_host <format index> <decoded.bin> <inputs.bin> <codes.bin>
// writes the FP32 value of every 16-bit code, then encodes the FP32 inputs;
// exits non-zero where a shortcut (zeros-run decoder, fixed-range encoder)
// differs from the general codec on its range.
// Format indices are the library's storage enum (FP16 2 ... P16_2C 7).
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "lbm_enc_table.h"

int main(int argc, char** argv) {
    if (argc != 5) return 2;
    const int fmt = std::atoi(argv[1]);
    std::vector<float> dec(65536);
    for (uint32_t c = 0; c < 65536; c++) dec[c] = lbm::decode16(fmt, c);
    // the sign-magnitude posits' shortcut for codes with a run of zeros as
    // regime (bit 14 clear) must equal the full decoder there, bit for bit
    if (fmt == lbm::S_P16_0S || fmt == lbm::S_P16_1S)
        for (uint32_t c = 0; c < 65536; c++) {
            if (c & 0x4000u) continue;
            const int32_t cs = (int32_t)(int16_t)(uint16_t)c;
            const float z = fmt == lbm::S_P16_0S ? lbm::posit_s_decode_zeros_run<0>(cs)
                                                 : lbm::posit_s_decode_zeros_run<1>(cs);
            if (lbm::f2u(z) != lbm::f2u(dec[c])) {
                std::fprintf(stderr, "zeros-run shortcut differs at code 0x%04x\n", c);
                return 8;
            }
        }
    FILE* f = std::fopen(argv[2], "wb");
    if (!f || std::fwrite(dec.data(), 4, dec.size(), f) != dec.size()) return 3;
    std::fclose(f);
    f = std::fopen(argv[3], "rb");
    if (!f) return 4;
    std::vector<float> in;
    float x;
    while (std::fread(&x, 4, 1, f) == 1) in.push_back(x);
    std::fclose(f);
    std::vector<uint16_t> out(in.size());
    if (fmt >= lbm::S_P16_0S) {
        std::vector<lbm::EncEntry> tab(lbm::kEncEntries);
        std::string why;
        if (!lbm::build_encoder_table(fmt, tab.data(), &why)) {
            std::fprintf(stderr, "table: %s\n", why.c_str());
            return 5;
        }
        for (size_t i = 0; i < in.size(); i++) out[i] = lbm::table_encode(in[i], tab.data(), lbm::enc_window_lo(fmt));
        // P16_0S's arithmetic encoder for |x| < 2^-7 must equal the table
        // encoder on every such float, both signs
        if (fmt == lbm::S_P16_0S)
            for (uint32_t u = 0; u < lbm::f2u(lbm::kP160sFixedBound); u++)
                for (uint32_t sg : {0u, 0x80000000u}) {
                    const float v = lbm::u2f(u | sg);
                    if (lbm::p160s_encode_fixed(v) != lbm::table_encode(v, tab.data(), lbm::enc_window_lo(fmt))) {
                        std::fprintf(stderr, "fixed-range encoder differs at 0x%08x\n", u | sg);
                        return 9;
                    }
                }
    } else if (fmt == lbm::S_FP16C) {
        for (size_t i = 0; i < in.size(); i++) out[i] = lbm::fp16c_encode(in[i]);
    } else {
        return 6;
    }
    f = std::fopen(argv[4], "wb");
    if (!f || std::fwrite(out.data(), 2, out.size(), f) != out.size()) return 7;
    std::fclose(f);
    return 0;
}
