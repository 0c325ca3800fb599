"""Mutation check of the oracle's pins: each case plants one plausible
mistake in a copy of oracle/lbm_oracle.c (a dropped term, a flipped sign or
direction, a wrong coefficient, a wrong codec constant), builds it on the
CPU, and runs the oracle's pin tests against that build in a subprocess.
Every mutant must make them fail; a mutant that passes would mean the
mistake it stands for is not pinned by anything.

CPU only: nothing here touches the GPU or the product library."""
import concurrent.futures as cf
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lbm_oracle.c")
PINS = [os.path.join(ROOT, "tests", "test_oracle_lbm.py"), os.path.join(ROOT, "tests", "test_oracle_codecs.py")]

# (name, text in lbm_oracle.c, replacement); the text must occur exactly once
MUTANTS = [
    ("force dropped from the velocity", "u_out[a] = (j + 0.5 * L->force[a]) / rho;", "u_out[a] = j / rho;"),
    ("pull from x + c_i", "const int sx = wrap(x - cv[i][0], L->nx);\n        const int sy = wrap(y - cv[i][1], L->ny);",
     "const int sx = wrap(x + cv[i][0], L->nx);\n        const int sy = wrap(y + cv[i][1], L->ny);"),
    ("shift 1 not added to rho", "if (L->shifted) rho += 1.0;", "(void)0;"),
    ("equilibrium B sign", "feq[i] = fma(w * rho, fma(0.5, fma(B, B, C), B), w * rhom1);",
     "feq[i] = fma(w * rho, fma(0.5, fma(B, B, C), -B), w * rhom1);"),
    ("equilibrium C factor", "const double C = -3.0 * (u[0] * u[0]", "const double C = -1.5 * (u[0] * u[0]"),
    ("moving wall sign", "v += 6.0 * weight(L->q, i) * 1.0 * cu;", "v -= 6.0 * weight(L->q, i) * 1.0 * cu;"),
    ("moving wall factor 3", "v += 6.0 * weight(L->q, i) * 1.0 * cu;", "v += 3.0 * weight(L->q, i) * 1.0 * cu;"),
    ("TRT rates swapped", "fo[i] = fi[i] - wp * (fp - ep) - wm * (fm - em);",
     "fo[i] = fi[i] - wm * (fp - ep) - wp * (fm - em);"),
    ("Guo antisymmetric sign", "*anti = w * 3.0 * cF;", "*anti = -w * 3.0 * cF;"),
    ("Guo second-moment coefficient", "*sym = w * (9.0 * cu * cF - 3.0 * uF);", "*sym = w * (4.5 * cu * cF - 3.0 * uF);"),
    ("Guo trace term", "*sym = w * (9.0 * cu * cF - 3.0 * uF);", "*sym = w * (9.0 * cu * cF - 1.5 * uF);"),
    ("Guo prefactor", "v += (1.0 - 0.5 * w) * (s + an);", "v += (s + an);"),
    ("clamp dropped", "for (int a = 0; a < 3; a++) u[a] = fmin(fmax(u[a], -cs), cs);", "(void)cs;"),
    ("clamp lets NaN through", "for (int a = 0; a < 3; a++) u[a] = fmin(fmax(u[a], -cs), cs);",
     "for (int a = 0; a < 3; a++) u[a] = u[a] < -cs ? -cs : (u[a] > cs ? cs : u[a]);"),
    ("non-finite cells not counted", "const int bad = !(isfinite(rho)", "const int bad = 0 && !(isfinite(rho)"),
    ("momentum exchange factor", "for (int a = 0; a < 3; a++) force[a] += cv[o][a] * (2.0 * fo + mv);",
     "for (int a = 0; a < 3; a++) force[a] += cv[o][a] * (1.0 * fo + mv);"),
    ("FP16C exponent bias", "ldexp((double)(2048 + m), e - 26);", "ldexp((double)(2048 + m), e - 25);"),
    ("posit regime offset", "const int r = first ? k - 1 : -k;", "const int r = first ? k : -k;"),
    ("P16_2C exponent offset", "return ldexp(1.0 + frac, -3 - 4 * r + e);", "return ldexp(1.0 + frac, -4 - 4 * r + e);"),
    ("ties to nearest even in FP16C", "else pick = ieee ? ((lo & 1) ? lo + 1 : lo) : lo + 1;",
     "else pick = (lo & 1) ? lo + 1 : lo;"),
    ("D3Q19 order: pairs 8 and 9 swapped",
     "{ 1,-1, 0}, {-1, 1, 0}, { 1, 0,-1}, {-1, 0, 1}, { 0, 1,-1}, { 0,-1, 1},\n    { 1, 1, 1}",
     "{ 1, 0,-1}, {-1, 0, 1}, { 1,-1, 0}, {-1, 1, 0}, { 0, 1,-1}, { 0,-1, 1},\n    { 1, 1, 1}"),
    ("D3Q19 weight", "case 19: { static const double w[3] = {1.0 / 3.0, 1.0 / 18.0, 1.0 / 36.0};",
     "case 19: { static const double w[3] = {1.0 / 3.0, 1.0 / 18.0, 1.0 / 30.0};"),
]


def _run_mutant(tmp_path, k, name, old, new, text):
    """Build mutant k and run the pins against it; returns (name, survived, tail)."""
    src = tmp_path / f"mutant{k}.c"
    src.write_text(text.replace(old, new))
    so = tmp_path / f"libmutant{k}.so"
    subprocess.run(["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                    "-o", str(so), str(src), "-lm"], check=True)
    env = dict(os.environ, LBM_ORACLE_SO=str(so), OMP_NUM_THREADS="2", OMP_WAIT_POLICY="passive")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *PINS],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    return name, r.returncode != 1, r.stdout[-1500:]


def test_every_mutant_is_caught_by_the_pins(tmp_path):
    text = open(SRC).read()
    for name, old, _ in MUTANTS:
        assert text.count(old) == 1, f"mutation site of '{name}' not found exactly once"
    with cf.ThreadPoolExecutor(4) as ex:
        results = list(ex.map(lambda a: _run_mutant(tmp_path, *a, text),
                              [(k, *m) for k, m in enumerate(MUTANTS)]))
    survivors = [(name, tail) for name, survived, tail in results if survived]
    assert not survivors, "mutants that survived the pins:\n" + "\n".join(f"{n}:\n{t}" for n, t in survivors)
