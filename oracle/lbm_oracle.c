/*
 * lbm_oracle.c -- plain FP64 CPU reference of the lattice Boltzmann step and of
 * the 16-bit storage formats of Lehmann et al., "On the accuracy and
 * performance of the lattice Boltzmann method with 64-bit, 32-bit and novel
 * 16-bit number formats" (arXiv 2112.08926).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is used by the test suite, by the smoke
 * check and by the CPU-baseline leg of the benchmark.  The product library
 * never links, loads or calls it, and it shares no code, header, table or
 * constant with the GPU path.
 *
 * It is deliberately slow and literal: one cell at a time, every step in the
 * order the paper states it, FP64 throughout.  OpenMP only splits the outer
 * z loop; it changes no arithmetic.
 *
 * Storage emulation: after collision each new DDF may be rounded to FP32 and
 * then passed through encode -> decode of a storage format, so that a run of
 * this oracle holds exactly the values a run with that storage would hold if
 * its arithmetic were exact.  The rounding decision (float -> code) is taken
 * from an FP32 value, as the paper's conversion routines take a float.
 *
 * Readings of the paper that this file relies on (the paper is silent or its
 * listings are inconsistent there) are marked READING in the comments.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Storage formats (Sec. 3, Table 2, Fig. 2)                                 */
/* ------------------------------------------------------------------------ */
enum {
    OF_FP64 = 0, OF_FP32 = 1, OF_FP16 = 2, OF_FP16S = 3, OF_FP16C = 4,
    OF_P16_0S = 5, OF_P16_1S = 6, OF_P16_2C = 7
};

/* IEEE-754 binary16: 1 sign | 5 exponent (bias 15) | 10 mantissa bits,
 * denormals at exponent 0, Inf/NaN at exponent 31 (Sec. 3.1.1, Table 2). */
static double ieee_half_value(uint32_t code)
{
    const int s = (code >> 15) & 1;
    const int e = (code >> 10) & 31;
    const int m = code & 1023;
    double v;
    if (e == 31) v = m ? NAN : INFINITY;
    else if (e == 0) v = ldexp((double)m, -24);              /* 2^-14 * m/2^10 */
    else v = ldexp((double)(1024 + m), e - 25);              /* 2^(e-15) * (1+m/2^10) */
    return s ? -v : v;
}

/* FP16C: 1 sign | 4 exponent (bias 15) | 11 mantissa bits, denormals at
 * exponent 0, no Inf/NaN: exponent 15 is an ordinary normal exponent
 * (Sec. 3.1.2 and 3.1.4, Table 2). */
static double fp16c_value(uint32_t code)
{
    const int s = (code >> 15) & 1;
    const int e = (code >> 11) & 15;
    const int m = code & 2047;
    const double v = (e == 0) ? ldexp((double)m, -25)       /* 2^-14 * m/2^11 */
                              : ldexp((double)(2048 + m), e - 26); /* 2^(e-15)*(1+m/2^11) */
    return s ? -v : v;
}

/* Posit with n_e exponent bits on the 15 magnitude bits of a sign-magnitude
 * 16-bit code (Sec. 3.2.1 and 3.2.3: sign bit instead of two's complement,
 * so there is a +0 and a -0 and no infinity).  The regime is the run of equal
 * bits that starts at the top magnitude bit; a run of k ones gives r = k-1,
 * a run of k zeros gives r = -k; the terminating bit follows.  Exponent bits
 * cut off by a long regime count as zero.  Value = (2^(2^n_e))^r * 2^e *
 * (1 + m/2^n_m). */
static double posit_magnitude(uint32_t mag, int n_e)
{
    if (mag == 0) return 0.0;
    const int first = (mag >> 14) & 1;
    int pos = 14, k = 0;
    while (pos >= 0 && (int)((mag >> pos) & 1) == first) { k++; pos--; }
    const int r = first ? k - 1 : -k;
    pos--;                                   /* skip the terminating bit */
    int e = 0;
    for (int j = 0; j < n_e; j++) {
        e <<= 1;
        if (pos >= 0) { e |= (mag >> pos) & 1; pos--; }
    }
    const int n_m = pos + 1;                 /* bits left for the mantissa */
    const double m = (n_m > 0) ? (double)(mag & ((1u << n_m) - 1)) : 0.0;
    const double frac = (n_m > 0) ? ldexp(m, -n_m) : 0.0;
    return ldexp(1.0 + frac, r * (1 << n_e) + e);
}

/* P16_2C, the asymmetric posit (Sec. 3.2.2): it only covers the lower flank,
 * so the regime is a run of r zeros closed by a one and has no sign bit of
 * its own; then 2 exponent bits and 12-r mantissa bits.
 * READING: value = 2^(-3 - 4r + e) * (1 + m/2^(12-r)); exponent bits cut off
 * by the regime are zero.  This gives 1.0 = 0x7000 (Fig. 2), the maximum
 * 1.999756 and the smallest value 2^-59 = 1.734724e-18 of Table 2. */
static double p162c_magnitude(uint32_t mag)
{
    if (mag == 0) return 0.0;
    int r = 0, pos = 14;
    while (((mag >> pos) & 1) == 0) { r++; pos--; }
    pos--;                                   /* skip the terminating one */
    int e = 0;
    for (int j = 0; j < 2; j++) {
        e <<= 1;
        if (pos >= 0) { e |= (mag >> pos) & 1; pos--; }
    }
    const int n_m = pos + 1;
    const double m = (n_m > 0) ? (double)(mag & ((1u << n_m) - 1)) : 0.0;
    const double frac = (n_m > 0) ? ldexp(m, -n_m) : 0.0;
    return ldexp(1.0 + frac, -3 - 4 * r + e);
}

/* Decoded value of a 16-bit storage code, by definition of the format.
 * FP16S and the two scaled posits undo their range shift here: FP16S stores
 * x*2^15 as FP16, P16_0S and P16_1S store x*2^7 as a posit (Listing 1 macros,
 * Sec. 3.1.2 and 3.2.2). */
double oracle_decode(int fmt, uint32_t code)
{
    code &= 0xFFFF;
    const double sgn = (code & 0x8000) ? -1.0 : 1.0;
    switch (fmt) {
    case OF_FP16:   return ieee_half_value(code);
    case OF_FP16S:  return ldexp(ieee_half_value(code), -15);
    case OF_FP16C:  return fp16c_value(code);
    case OF_P16_0S: return sgn * ldexp(posit_magnitude(code & 0x7FFF, 0), -7);
    case OF_P16_1S: return sgn * ldexp(posit_magnitude(code & 0x7FFF, 1), -7);
    case OF_P16_2C: return sgn * p162c_magnitude(code & 0x7FFF);
    default:        return NAN;
    }
}

/* Sorted table of the non-negative finite values of each 16-bit format,
 * indexed by magnitude code.  Every format here is monotone in its magnitude
 * code, which the tests check exhaustively. */
static double g_table[8][32768];
static int g_table_len[8];
static int g_table_ready[8];

static void build_table(int fmt)
{
    if (g_table_ready[fmt]) return;
    int len = 0;
    for (uint32_t c = 0; c < 32768; c++) {
        const double v = oracle_decode(fmt, c);
        if (!isfinite(v)) break;             /* FP16: 0x7C00 is +Inf */
        g_table[fmt][len++] = v;
    }
    g_table_len[fmt] = len;
    g_table_ready[fmt] = 1;
}

/* Code of a float in a 16-bit format.
 * FP16 and FP16S: IEEE round-to-nearest-even (hardware conversion,
 * Sec. 3.1.3), FP16S on x*2^15; magnitudes at or above 65520 (after scaling)
 * overflow to Inf, NaN stays NaN.
 * FP16C and the posits.  READING: nearest representable value, ties to the
 * larger magnitude; magnitudes above the largest value (including Inf) give
 * the largest value (the optional saturation of Sec. 3.1.4); NaN gives the
 * largest value with the NaN's sign bit; the scaled posits round x*2^7. */
uint32_t oracle_encode(int fmt, float xf)
{
    const uint32_t sign = signbit(xf) ? 0x8000u : 0u;
    build_table(fmt);
    const double *t = g_table[fmt];
    const int len = g_table_len[fmt];
    const int ieee = (fmt == OF_FP16 || fmt == OF_FP16S);
    if (isnan(xf)) return sign | (ieee ? 0x7E00u : 0x7FFFu);
    /* |x| in the units of the table; scaling by a power of two is exact */
    double a = fabs((double)xf);
    if (ieee) {
        double h = (fmt == OF_FP16S) ? a * 32768.0 : a;
        if (h >= 65520.0) return sign | 0x7C00u;   /* rounds past 65504 -> Inf */
        a = ldexp(h, fmt == OF_FP16S ? -15 : 0);
    }
    if (isinf(a) || a >= t[len - 1]) return sign | (uint32_t)(len - 1);
    /* largest lo with t[lo] <= a */
    int lo = 0, hi = len - 1;
    while (hi - lo > 1) {
        const int mid = (lo + hi) / 2;
        if (t[mid] <= a) lo = mid; else hi = mid;
    }
    if (t[lo] == a) return sign | (uint32_t)lo;
    /* t[lo] < a < t[lo+1]; both differences are exact in double */
    const double below = a - t[lo], above = t[lo + 1] - a;
    int pick;
    if (below < above) pick = lo;
    else if (above < below) pick = lo + 1;
    else pick = ieee ? ((lo & 1) ? lo + 1 : lo) : lo + 1;
    return sign | (uint32_t)pick;
}

/* Value a DDF holds after being stored in format fmt: FP64 keeps it, FP32
 * rounds it to float, a 16-bit format rounds it to float and then to the
 * nearest code as above. */
static double stored_value(int fmt, double v)
{
    if (fmt == OF_FP64) return v;
    const float f = (float)v;
    if (fmt == OF_FP32) return (double)f;
    return oracle_decode(fmt, oracle_encode(fmt, f));
}

void oracle_encode_array(int fmt, const float *x, uint16_t *out, int64_t n)
{
    for (int64_t k = 0; k < n; k++) out[k] = (uint16_t)oracle_encode(fmt, x[k]);
}

void oracle_decode_array(int fmt, const uint16_t *codes, double *out, int64_t n)
{
    for (int64_t k = 0; k < n; k++) out[k] = oracle_decode(fmt, codes[k]);
}

void oracle_store_array(int fmt, const double *v, double *out, int64_t n)
{
    for (int64_t k = 0; k < n; k++) out[k] = stored_value(fmt, v[k]);
}

/* ------------------------------------------------------------------------ */
/* Velocity sets (Sec. 2.1, Listing 2, Table 1)                             */
/* ------------------------------------------------------------------------ */
/* D3Q19 in the order of the neighbour list of Listing 2: 0 rest, then the
 * opposite pairs +00 -00, 0+0 0-0, 00+ 00-, ++0 --0, +0+ -0-, 0++ 0--,
 * +-0 -+0, +0- -0+, 0+- 0-+.  Weights 1/3, 1/18, 1/36 (Sec. 2.3).
 * READING for D3Q27 (its table is only cited): the 19 above, then the corner
 * pairs +++ ---, ++- --+, +-+ -+-, -++ +--; weights 8/27, 2/27, 1/54,
 * 1/216.  Table 1's delta values for D3Q27 come out only with these weights,
 * which the tests check. */
static const int C27[27][3] = {
    { 0, 0, 0},
    { 1, 0, 0}, {-1, 0, 0}, { 0, 1, 0}, { 0,-1, 0}, { 0, 0, 1}, { 0, 0,-1},
    { 1, 1, 0}, {-1,-1, 0}, { 1, 0, 1}, {-1, 0,-1}, { 0, 1, 1}, { 0,-1,-1},
    { 1,-1, 0}, {-1, 1, 0}, { 1, 0,-1}, {-1, 0, 1}, { 0, 1,-1}, { 0,-1, 1},
    { 1, 1, 1}, {-1,-1,-1}, { 1, 1,-1}, {-1,-1, 1}, { 1,-1, 1}, {-1, 1,-1},
    {-1, 1, 1}, { 1,-1,-1}
};
/* READING for the other sets of Table 1 (only named there): the same
 * conventions (rest first, then opposite pairs), the directions in the
 * D3Q19/D3Q27 order restricted to the set.  D2Q9: the four axis directions
 * in x and y and the four xy diagonals, weights 4/9, 1/9, 1/36.  D3Q7: rest
 * and the six faces, weights 1/4, 1/8.  D3Q13: rest and the twelve edge
 * directions, weights 1/2, 1/24.  D3Q15: rest, six faces, eight corners,
 * weights 2/9, 1/9, 1/72.  Table 1's delta values of all four come out only
 * with these weights and the equilibrium of Sec. 2.2 (checked by the tests). */
static const int C9[9][3] = {
    { 0, 0, 0}, { 1, 0, 0}, {-1, 0, 0}, { 0, 1, 0}, { 0,-1, 0},
    { 1, 1, 0}, {-1,-1, 0}, { 1,-1, 0}, {-1, 1, 0}
};
static const int C13[13][3] = {
    { 0, 0, 0},
    { 1, 1, 0}, {-1,-1, 0}, { 1, 0, 1}, {-1, 0,-1}, { 0, 1, 1}, { 0,-1,-1},
    { 1,-1, 0}, {-1, 1, 0}, { 1, 0,-1}, {-1, 0, 1}, { 0, 1,-1}, { 0,-1, 1}
};
static const int C15[15][3] = {
    { 0, 0, 0},
    { 1, 0, 0}, {-1, 0, 0}, { 0, 1, 0}, { 0,-1, 0}, { 0, 0, 1}, { 0, 0,-1},
    { 1, 1, 1}, {-1,-1,-1}, { 1, 1,-1}, {-1,-1, 1}, { 1,-1, 1}, {-1, 1,-1},
    {-1, 1, 1}, { 1,-1,-1}
};

static int valid_q(int q) { return q == 7 || q == 9 || q == 13 || q == 15 || q == 19 || q == 27; }

/* direction table of a velocity set (D3Q7 and D3Q19 are prefixes of D3Q27) */
static const int (*velocities(int q))[3]
{
    switch (q) {
    case 9:  return C9;
    case 13: return C13;
    case 15: return C15;
    default: return C27;
    }
}

/* weight by the squared length of c_i */
static double weight(int q, int i)
{
    const int (*C)[3] = velocities(q);
    const int len2 = C[i][0] * C[i][0] + C[i][1] * C[i][1] + C[i][2] * C[i][2];
    switch (q) {
    case 7:  return len2 == 0 ? 1.0 / 4.0 : 1.0 / 8.0;
    case 9:  { static const double w[3] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 36.0}; return w[len2]; }
    case 13: return len2 == 0 ? 1.0 / 2.0 : 1.0 / 24.0;
    case 15: { static const double w[4] = {2.0 / 9.0, 1.0 / 9.0, 0.0, 1.0 / 72.0}; return w[len2]; }
    case 19: { static const double w[3] = {1.0 / 3.0, 1.0 / 18.0, 1.0 / 36.0}; return w[len2]; }
    default: { static const double w[4] = {8.0 / 27.0, 2.0 / 27.0, 1.0 / 54.0, 1.0 / 216.0}; return w[len2]; }
    }
}

/* opposite direction: pairs are (2k-1, 2k) */
static int opposite(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

int oracle_velset(int q, int32_t *c, double *w, int32_t *opp)
{
    if (!valid_q(q)) return -1;
    const int (*C)[3] = velocities(q);
    for (int i = 0; i < q; i++) {
        for (int a = 0; a < 3; a++) c[3 * i + a] = C[i][a];
        w[i] = weight(q, i);
        opp[i] = opposite(i);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Equilibrium (Sec. 2.2, shifted form and its 3-FMA evaluation order;      */
/* appendix "LBM equations in a nutshell" for the unshifted form)           */
/* ------------------------------------------------------------------------ */
/* Shifted: feq_i - w_i = w_i rho (1/2 (B^2 + C) + B) + w_i (rho - 1) with
 * B = 3 u.c_i and C = -3 u.u, i.e. three FMAs per direction once A = w_i rho
 * and D = w_i (rho - 1) are formed.  Unshifted: w_i rho (1/2 (B^2+C) + B + 1). */
void oracle_equilibrium(int q, int shifted, double rho, const double *u, double *feq)
{
    const int (*cv)[3] = velocities(q);
    const double C = -3.0 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    const double rhom1 = rho - 1.0;
    for (int i = 0; i < q; i++) {
        const double w = weight(q, i);
        const double B = 3.0 * (u[0] * cv[i][0] + u[1] * cv[i][1] + u[2] * cv[i][2]);
        if (shifted)
            feq[i] = fma(w * rho, fma(0.5, fma(B, B, C), B), w * rhom1);
        else
            feq[i] = w * rho * (0.5 * (B * B + C) + B + 1.0);
    }
}

/* ------------------------------------------------------------------------ */
/* Lattice and one time step (appendix: streaming, fields, equilibrium,      */
/* collision; Listing 2 for order, bounce-back and the velocity clamp)       */
/* ------------------------------------------------------------------------ */
enum { OFLAG_SOLID = 1, OFLAG_EQ = 2, OFLAG_MOVING = 4 };

typedef struct {
    int32_t nx, ny, nz, q;
    int32_t collision;     /* 0 SRT (BGK), 1 TRT, 2 MRT (D3Q19) */
    int32_t storage;       /* emulated storage format of the new DDFs */
    int32_t shifted;       /* 1: the DDFs are f_i - w_i (Sec. 2.2) */
    int32_t nthreads;      /* OpenMP threads for the z loop (0: default) */
    double omega;          /* 1/tau; for TRT the symmetric rate omega+ */
    double omega_minus;    /* TRT antisymmetric rate (ignored for SRT) */
    double force[3];       /* Guo body force per volume */
    double wall_u[3];      /* velocity of MOVING wall cells (rho_w = 1) */
    double mrt_rates[19];  /* MRT: relaxation rate of each moment (D3Q19) */
} oracle_lattice;

static inline int64_t cell(const oracle_lattice *L, int x, int y, int z)
{
    return (int64_t)x + (int64_t)L->nx * ((int64_t)y + (int64_t)L->ny * z);
}

static inline int wrap(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

/* Streaming (pull): the DDF moving along c_i arrives at x from x - c_i, with
 * periodic wrap at the box faces (Listing 2 neighbour list).  If that source
 * cell is a wall, the DDF is the one that left x towards the wall in the
 * previous step, f_opp(i)(x) (mid-grid bounce-back).  READING for moving walls
 * (only cited in the paper): the reflected DDF gains 6 w_i rho_w (c_i . u_w)
 * with rho_w = 1; this term is the same with and without shifting. */
static void pull(const oracle_lattice *L, const double *f, const uint8_t *flags,
                 int x, int y, int z, double *fi)
{
    const int64_t N = (int64_t)L->nx * L->ny * L->nz;
    const int64_t n = cell(L, x, y, z);
    const int (*cv)[3] = velocities(L->q);
    for (int i = 0; i < L->q; i++) {
        const int sx = wrap(x - cv[i][0], L->nx);
        const int sy = wrap(y - cv[i][1], L->ny);
        const int sz = wrap(z - cv[i][2], L->nz);
        const int64_t s = cell(L, sx, sy, sz);
        if (flags[s] & OFLAG_SOLID) {
            double v = f[(int64_t)opposite(i) * N + n];
            if (flags[s] & OFLAG_MOVING) {
                const double cu = cv[i][0] * L->wall_u[0] + cv[i][1] * L->wall_u[1]
                                + cv[i][2] * L->wall_u[2];
                v += 6.0 * weight(L->q, i) * 1.0 * cu;
            }
            fi[i] = v;
        } else {
            fi[i] = f[(int64_t)i * N + s];
        }
    }
}

/* Density and momentum (Sec. 2.2 and Listing 2): rho is f_0 + f_1 + ... in
 * index order with the 1 of the shift added last; each momentum component is
 * summed over the opposite pairs in index order with alternating signs.
 * READING for the Guo force (only cited): u = (sum_i c_i f_i + F/2) / rho. */
static void fields(const oracle_lattice *L, const double *fi, double *rho_out, double *u_out)
{
    const int (*cv)[3] = velocities(L->q);
    double rho = fi[0];
    for (int i = 1; i < L->q; i++) rho += fi[i];
    if (L->shifted) rho += 1.0;
    for (int a = 0; a < 3; a++) {
        double j = 0.0;
        for (int i = 1; i < L->q; i += 2) {
            const int c = cv[i][a];
            if (c > 0) { j += fi[i]; j -= fi[i + 1]; }
            else if (c < 0) { j += fi[i + 1]; j -= fi[i]; }
        }
        u_out[a] = (j + 0.5 * L->force[a]) / rho;
    }
    *rho_out = rho;
}

/* Guo source term split into its part symmetric under i <-> opp(i),
 * w_i (9 (c_i.u)(c_i.F) - 3 u.F), and its antisymmetric part w_i 3 c_i.F.
 * READING: SRT adds (1 - omega/2) times their sum (Guo's scheme); TRT scales
 * the symmetric part by (1 - omega+/2) and the antisymmetric one by
 * (1 - omega-/2), which reduces to SRT when both rates are equal. */
static void guo_parts(const oracle_lattice *L, int i, const double *u, double *sym, double *anti)
{
    const double *F = L->force;
    const int (*cv)[3] = velocities(L->q);
    const double cF = cv[i][0] * F[0] + cv[i][1] * F[1] + cv[i][2] * F[2];
    const double cu = cv[i][0] * u[0] + cv[i][1] * u[1] + cv[i][2] * u[2];
    const double uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
    const double w = weight(L->q, i);
    *sym = w * (9.0 * cu * cF - 3.0 * uF);
    *anti = w * 3.0 * cF;
}

/* READING for MRT (named in Sec. 2.1 and in the roofline of Sec. 5, not
 * defined in the paper): the D3Q19 moment basis of d'Humieres et al. (2002),
 * each moment a polynomial in c_i with c2 = |c_i|^2:
 *   rho 1; e 19 c2 - 30; eps (21 c2^2 - 53 c2 + 24)/2;
 *   j_a c_a and q_a (5 c2 - 9) c_a for a = x, y, z (interleaved j, q);
 *   3p_xx 3 cx^2 - c2; 3pi_xx (3 c2 - 5)(3 cx^2 - c2);
 *   p_ww cy^2 - cz^2; pi_ww (3 c2 - 5)(cy^2 - cz^2);
 *   p_xy cx cy, p_yz cy cz, p_xz cx cz;
 *   m_x (cy^2 - cz^2) cx, m_y (cz^2 - cx^2) cy, m_z (cx^2 - cy^2) cz.
 * The rows are orthogonal, so M^-1 = M^T diag(1/|row|^2).  The collision
 * relaxes the non-equilibrium moments M (f - f^eq) with the rates s_k (the
 * equilibrium moments are those of the Sec. 2.2 equilibrium, M f^eq) and adds
 * the Guo source in moment space scaled by (1 - s_k/2):
 *   f' = f - M^-1 [ S M (f - f^eq) - (I - S/2) M S^F ].
 * With every s_k equal to omega this is the SRT step.  Shifting drops out of
 * f - f^eq. */
static void mrt_basis(double M[19][19], double norm2[19])
{
    for (int i = 0; i < 19; i++) {
        const double cx = C27[i][0], cy = C27[i][1], cz = C27[i][2];
        const double c2 = cx * cx + cy * cy + cz * cz;
        const double row[19] = {
            1.0, 19.0 * c2 - 30.0, (21.0 * c2 * c2 - 53.0 * c2 + 24.0) / 2.0,
            cx, (5.0 * c2 - 9.0) * cx, cy, (5.0 * c2 - 9.0) * cy, cz, (5.0 * c2 - 9.0) * cz,
            3.0 * cx * cx - c2, (3.0 * c2 - 5.0) * (3.0 * cx * cx - c2),
            cy * cy - cz * cz, (3.0 * c2 - 5.0) * (cy * cy - cz * cz),
            cx * cy, cy * cz, cx * cz,
            (cy * cy - cz * cz) * cx, (cz * cz - cx * cx) * cy, (cx * cx - cy * cy) * cz};
        for (int k = 0; k < 19; k++) M[k][i] = row[k];
    }
    for (int k = 0; k < 19; k++) {
        norm2[k] = 0.0;
        for (int i = 0; i < 19; i++) norm2[k] += M[k][i] * M[k][i];
    }
}

void oracle_mrt_basis(double *M, double *norm2)
{
    double m[19][19];
    mrt_basis(m, norm2);
    for (int k = 0; k < 19; k++)
        for (int i = 0; i < 19; i++) M[19 * k + i] = m[k][i];
}

static void collide_mrt(const oracle_lattice *L, const double *fi, const double *feq, const double *u,
                        int forced, double *fo)
{
    double M[19][19], n2[19], r[19], src[19];
    mrt_basis(M, n2);
    for (int i = 0; i < 19; i++) {
        double s = 0.0, an = 0.0;
        if (forced) guo_parts(L, i, u, &s, &an);
        src[i] = s + an;
    }
    for (int k = 0; k < 19; k++) {
        double m = 0.0, g = 0.0;
        for (int i = 0; i < 19; i++) {
            m += M[k][i] * (fi[i] - feq[i]);
            g += M[k][i] * src[i];
        }
        r[k] = L->mrt_rates[k] * m - (1.0 - 0.5 * L->mrt_rates[k]) * g;
    }
    for (int i = 0; i < 19; i++) {
        double d = 0.0;
        for (int k = 0; k < 19; k++) d += M[k][i] * r[k] / n2[k];
        fo[i] = fi[i] - d;
    }
}

/* Collides one cell; returns 1 if its density or a velocity component, as
 * computed from the pulled DDFs before the clamp, is not finite (a blow-up
 * that the clamp and the saturating 16-bit encoders would otherwise hide),
 * else 0.
 * The clamp is the listing's OpenCL clamp(u, -c, c), which that language
 * defines as fmin(fmax(u, -c), c); fmin and fmax return the other operand
 * when one is NaN, so a NaN component becomes -c.  C's fmin/fmax have the
 * same rule. */
static int collide_cell(const oracle_lattice *L, const double *fi, double *fo)
{
    double rho, u[3], feq[27];
    fields(L, fi, &rho, u);
    const int bad = !(isfinite(rho) && isfinite(u[0]) && isfinite(u[1]) && isfinite(u[2]));
    const double cs = 1.0 / sqrt(3.0);           /* lattice speed of sound */
    for (int a = 0; a < 3; a++) u[a] = fmin(fmax(u[a], -cs), cs);
    oracle_equilibrium(L->q, L->shifted, rho, u, feq);
    const int forced = (L->force[0] != 0.0 || L->force[1] != 0.0 || L->force[2] != 0.0);
    const double w = L->omega;
    if (L->collision == 2) {
        collide_mrt(L, fi, feq, u, forced, fo);
    } else if (L->collision == 0) {
        /* SRT / BGK: f' = (1 - 1/tau) f + (1/tau) feq, as one FMA */
        for (int i = 0; i < L->q; i++) {
            double v = fma(1.0 - w, fi[i], w * feq[i]);
            if (forced) {
                double s, an;
                guo_parts(L, i, u, &s, &an);
                v += (1.0 - 0.5 * w) * (s + an);
            }
            fo[i] = v;
        }
    } else {
        /* READING for TRT (only named): relax the symmetric and antisymmetric
         * parts of each opposite pair with omega+ and omega-. */
        const double wp = w, wm = L->omega_minus;
        fo[0] = fi[0] - wp * (fi[0] - feq[0]);
        if (forced) {
            double s, an;
            guo_parts(L, 0, u, &s, &an);
            fo[0] += (1.0 - 0.5 * wp) * s + (1.0 - 0.5 * wm) * an;
        }
        for (int i = 1; i < L->q; i += 2) {
            const int k = i + 1;
            const double fp = 0.5 * (fi[i] + fi[k]), fm = 0.5 * (fi[i] - fi[k]);
            const double ep = 0.5 * (feq[i] + feq[k]), em = 0.5 * (feq[i] - feq[k]);
            fo[i] = fi[i] - wp * (fp - ep) - wm * (fm - em);
            fo[k] = fi[k] - wp * (fp - ep) + wm * (fm - em);
            if (forced) {
                double s, an;
                guo_parts(L, i, u, &s, &an);
                fo[i] += (1.0 - 0.5 * wp) * s + (1.0 - 0.5 * wm) * an;
                guo_parts(L, k, u, &s, &an);
                fo[k] += (1.0 - 0.5 * wp) * s + (1.0 - 0.5 * wm) * an;
            }
        }
    }
    return bad;
}

/* One time step fin -> fout, both [q][N] with cell index n = x + (y + z ny) nx.
 * Wall (SOLID) cells are skipped as in Listing 2 and keep their content;
 * READING for equilibrium (EQ) cells (only cited): they hold the equilibrium
 * of their fixed density and velocity and are not updated either.
 * Returns -1 for an unsupported lattice, else the number of fluid cells
 * whose density or velocity before the clamp was not finite. */
int64_t oracle_step(const oracle_lattice *L, const double *fin, double *fout, const uint8_t *flags)
{
    if (!valid_q(L->q)) return -1;
    if (L->collision == 2 && L->q != 19) return -1;     /* the MRT basis is D3Q19's */
    const int64_t N = (int64_t)L->nx * L->ny * L->nz;
    if (L->storage >= OF_FP16) build_table(L->storage);   /* before the threads start */
    int64_t nonfinite = 0;
#ifdef _OPENMP
    const int nt = L->nthreads > 0 ? L->nthreads : 0;
#pragma omp parallel for schedule(static) num_threads(nt > 0 ? nt : omp_get_max_threads()) reduction(+ : nonfinite)
#endif
    for (int z = 0; z < L->nz; z++) {
        double fi[27], fo[27];
        for (int y = 0; y < L->ny; y++)
            for (int x = 0; x < L->nx; x++) {
                const int64_t n = cell(L, x, y, z);
                if (flags[n] & (OFLAG_SOLID | OFLAG_EQ)) {
                    for (int i = 0; i < L->q; i++) fout[(int64_t)i * N + n] = fin[(int64_t)i * N + n];
                    continue;
                }
                pull(L, fin, flags, x, y, z, fi);
                nonfinite += collide_cell(L, fi, fo);
                for (int i = 0; i < L->q; i++)
                    fout[(int64_t)i * N + n] = stored_value(L->storage, fo[i]);
            }
    }
    return nonfinite;
}

/* Density and velocity the next step would see at every cell: pull, then
 * the sums of fields() (velocity not clamped).  Wall cells report rho = 1 and
 * the wall velocity (zero unless MOVING); EQ cells report rho and u of their
 * stored equilibrium, i.e. the moments of their own DDFs. */
int oracle_moments(const oracle_lattice *L, const double *f, const uint8_t *flags,
                   double *rho, double *u)
{
    const int64_t N = (int64_t)L->nx * L->ny * L->nz;
    for (int z = 0; z < L->nz; z++)
        for (int y = 0; y < L->ny; y++)
            for (int x = 0; x < L->nx; x++) {
                const int64_t n = cell(L, x, y, z);
                double fi[27], r, uu[3];
                if (flags[n] & OFLAG_SOLID) {
                    const int mv = (flags[n] & OFLAG_MOVING) != 0;
                    rho[n] = 1.0;
                    for (int a = 0; a < 3; a++) u[a * N + n] = mv ? L->wall_u[a] : 0.0;
                    continue;
                }
                if (flags[n] & OFLAG_EQ) {
                    oracle_lattice L0 = *L;
                    L0.force[0] = L0.force[1] = L0.force[2] = 0.0;
                    for (int i = 0; i < L->q; i++) fi[i] = f[(int64_t)i * N + n];
                    fields(&L0, fi, &r, uu);
                } else {
                    pull(L, f, flags, x, y, z, fi);
                    fields(L, fi, &r, uu);
                }
                rho[n] = r;
                for (int a = 0; a < 3; a++) u[a * N + n] = uu[a];
            }
    return 0;
}

/* DDFs of the equilibrium of given fields (the paper's initialize kernel),
 * passed through the storage format.  Wall cells hold zeros (READING: the
 * paper never writes them; zero keeps runs deterministic). */
int oracle_init(const oracle_lattice *L, const double *rho, const double *u,
                const uint8_t *flags, double *f)
{
    const int64_t N = (int64_t)L->nx * L->ny * L->nz;
    for (int64_t n = 0; n < N; n++) {
        double feq[27], uu[3] = {u[n], u[N + n], u[2 * N + n]};
        if (flags[n] & OFLAG_SOLID) {
            for (int i = 0; i < L->q; i++) f[(int64_t)i * N + n] = 0.0;
            continue;
        }
        oracle_equilibrium(L->q, L->shifted, rho[n], uu, feq);
        for (int i = 0; i < L->q; i++) f[(int64_t)i * N + n] = stored_value(L->storage, feq[i]);
    }
    return 0;
}

/* FP64 diagnostics over the fluid cells (not SOLID, not EQ), in cell order:
 * out[0] mass sum rho, out[1..3] momentum sum rho u, out[4] kinetic energy
 * sum rho |u|^2 / 2 (Sec. 4.2), out[5] max |u|, out[6] relative L2 velocity
 * error against u_ref (Sec. 4.1 error norm; -1 without u_ref), out[7..9]
 * force on the walls by momentum exchange, out[10] number of fluid cells with
 * a non-finite rho or u.
 * READING for the force (not in the paper): each fluid-to-wall link with wall
 * source x - c_i carries c_opp(i) (2 (f_opp(i)(x) + w) + 6 w_i rho_w c_i.u_w)
 * into the wall (w is the weight when the DDFs are shifted, else 0). */
int oracle_diagnostics(const oracle_lattice *L, const double *f, const uint8_t *flags,
                       const double *u_ref, double *out)
{
    const int64_t N = (int64_t)L->nx * L->ny * L->nz;
    double mass = 0, mom[3] = {0, 0, 0}, ke = 0, umax = 0, err2 = 0, ref2 = 0, force[3] = {0, 0, 0};
    double nonfinite = 0;
    for (int z = 0; z < L->nz; z++)
        for (int y = 0; y < L->ny; y++)
            for (int x = 0; x < L->nx; x++) {
                const int64_t n = cell(L, x, y, z);
                if (flags[n] & (OFLAG_SOLID | OFLAG_EQ)) continue;
                double fi[27], r, u[3];
                pull(L, f, flags, x, y, z, fi);
                fields(L, fi, &r, u);
                if (!isfinite(r) || !isfinite(u[0]) || !isfinite(u[1]) || !isfinite(u[2])) {
                    nonfinite += 1.0;
                    continue;
                }
                mass += r;
                for (int a = 0; a < 3; a++) mom[a] += r * u[a];
                const double u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
                ke += 0.5 * r * u2;
                if (sqrt(u2) > umax) umax = sqrt(u2);
                if (u_ref) {
                    for (int a = 0; a < 3; a++) {
                        const double d = u[a] - u_ref[a * N + n];
                        err2 += d * d;
                        ref2 += u_ref[a * N + n] * u_ref[a * N + n];
                    }
                }
                const int (*cv)[3] = velocities(L->q);
                for (int i = 1; i < L->q; i++) {
                    const int sx = wrap(x - cv[i][0], L->nx);
                    const int sy = wrap(y - cv[i][1], L->ny);
                    const int sz = wrap(z - cv[i][2], L->nz);
                    const int64_t s = cell(L, sx, sy, sz);
                    if (!(flags[s] & OFLAG_SOLID)) continue;
                    const int o = opposite(i);
                    const double fo = f[(int64_t)o * N + n] + (L->shifted ? weight(L->q, o) : 0.0);
                    double mv = 0.0;
                    if (flags[s] & OFLAG_MOVING)
                        mv = 6.0 * weight(L->q, i) * (cv[i][0] * L->wall_u[0] + cv[i][1] * L->wall_u[1]
                                                      + cv[i][2] * L->wall_u[2]);
                    for (int a = 0; a < 3; a++) force[a] += cv[o][a] * (2.0 * fo + mv);
                }
            }
    out[0] = mass;
    for (int a = 0; a < 3; a++) out[1 + a] = mom[a];
    out[4] = ke;
    out[5] = umax;
    out[6] = u_ref ? (ref2 > 0 ? sqrt(err2 / ref2) : 0.0) : -1.0;
    for (int a = 0; a < 3; a++) out[7 + a] = force[a];
    out[10] = nonfinite;
    return 0;
}
