"""Writes tests/golden/poiseuille_sweep_errors.txt with the FP64 reference
(oracle/ only): the Poiseuille radius sweep of Sec. 4.1 (its figure of the
error E against the radius R at constant Reynolds number and centre
velocity) at the three smallest radii, R = 8, 16, 32: Re = 2 R u_max / nu =
10, u_max = 0.1, D3Q19 SRT, Guo force 4 nu u_max / R^2, mid-grid bounce-back
in a cylinder, channel along the periodic axis with Lx = 1 (every slice is
the same), 3 R^2 / nu steps from rest (rounded up to a multiple of 100), with
each storage format emulated on the stored DDFs (FP64 arithmetic).  One line
per radius and format: the relative L2 error E against the parabola and the
largest velocity.

    python tests/golden/make_poiseuille_sweep.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle                     # noqa: E402
import lbm_workloads as wl        # noqa: E402

RE, UMAX = 10.0, 0.1
RADII = (8, 16, 32)
FORMATS = ["fp64", "fp32", "fp16", "fp16s", "fp16c", "p16_0s", "p16_1s", "p16_2c"]


def case(R):
    nu = 2 * R * UMAX / RE
    tau = 3 * nu + 0.5
    force = 4 * nu * UMAX / R ** 2
    steps = int(3 * R * R / nu) // 100 * 100 + 100
    return nu, tau, force, steps


def main():
    lines = [f"# R  format  E_L2_vs_parabola  u_max   (FP64 reference, storage emulated; Re={RE} u_max={UMAX}, "
             "tau = 3 nu + 1/2, steps = 3 R^2/nu rounded up to 100)"]
    for R in RADII:
        nu, tau, force, steps = case(R)
        ny = 2 * (R + 1)
        flags = wl.poiseuille_flags(1, ny, ny, R)
        u_ref = wl.poiseuille_profile(1, ny, ny, R, force, nu)
        for fmt in FORMATS:
            lat = oracle.Lattice(1, ny, ny, q=19, tau=tau, force=(force, 0, 0), flags=flags, storage=fmt).init()
            lat.step(steps)
            d = lat.diagnostics(u_ref)
            lines.append(f"{R:3d} {fmt:8s} {d['l2_error']:.9e} {d['u_max']:.9e}")
            print(lines[-1], flush=True)
    with open(os.path.join(HERE, "poiseuille_sweep_errors.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
