"""Writes tests/golden/poiseuille_r31_errors.txt with the FP64 reference
(oracle/ only): steady Poiseuille flow through a cylinder of radius R = 31
(Sec. 4.1; channel along the periodic axis, Lx = 1 since every x slice is the
same), D3Q19 SRT, tau 0.8, Guo force 1e-6, 50 000 steps from rest, with each
storage format emulated on the stored DDFs; one line per format with the L2
error E against the parabola and the largest velocity; the lines
"<format>_unshifted" are the same run without DDF shifting (Sec. 2.2
ablation: the DDFs stored as f_i).

    python tests/golden/make_poiseuille_errors.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle                     # noqa: E402
import lbm_workloads as wl        # noqa: E402

R, TAU, F, STEPS, NY = 31, 0.8, 1e-6, 50000, 64


def main():
    nu = (TAU - 0.5) / 3.0
    flags = wl.poiseuille_flags(1, NY, NY, R)
    u_ref = wl.poiseuille_profile(1, NY, NY, R, F, nu)
    lines = ["# format  E_L2_vs_parabola  u_max   (FP64 reference, storage emulated; "
             f"R={R} tau={TAU} F={F} steps={STEPS})"]
    runs = [(f, True) for f in ["fp64", "fp32", "fp16", "fp16s", "fp16c", "p16_0s", "p16_1s", "p16_2c"]]
    runs += [(f, False) for f in ["fp32", "fp16s", "fp16c"]]
    for fmt, shifted in runs:
        lat = oracle.Lattice(1, NY, NY, q=19, tau=TAU, force=(F, 0, 0), flags=flags, storage=fmt,
                             shifted=shifted).init()
        lat.step(STEPS)
        d = lat.diagnostics(u_ref)
        name = fmt if shifted else fmt + "_unshifted"
        lines.append(f"{name:16s} {d['l2_error']:.6e} {d['u_max']:.6e}")
        print(lines[-1], flush=True)
    with open(os.path.join(HERE, "poiseuille_r31_errors.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
