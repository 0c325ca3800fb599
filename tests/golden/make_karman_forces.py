"""Writes tests/golden/karman_reduced_forces.txt with the FP64 reference
(oracle/ only): the Karman vortex street of Sec. 4.3 in 3-D at reduced size
256 x 64 x 16 (flow along +x, cylinder of radius 4 along z centred at
(64, 32), equilibrium cells with rho 1, u (0.05, 0, 0) on the x and y faces,
periodic in z, velocity 0.05 on the half y < 32 at the start), D3Q27 TRT
(magic 1/4), tau 0.548; force on the cylinder by momentum exchange every
250 steps up to 5000.

    python tests/golden/make_karman_forces.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle                     # noqa: E402
import lbm_workloads as wl        # noqa: E402

NX, NY, NZ, R, CX, CY, U0, TAU, STEPS, EVERY = 256, 64, 16, 4.0, 64.0, 32.0, 0.05, 0.548, 5000, 250


def main():
    flags = wl.karman_flags(NX, NY, NZ, R, CX, CY)
    rho, u = wl.karman_fields(NX, NY, NZ, U0)
    eq = (flags & wl.EQ) != 0
    u[:, eq] = 0.0
    u[0, eq] = U0
    rho[eq] = 1.0
    lat = oracle.Lattice(NX, NY, NZ, q=27, tau=TAU, collision="trt", flags=flags).init(rho, u)
    lines = [f"# step Fx Fy Fz  (FP64 reference; {NX}x{NY}x{NZ} D3Q27 TRT tau={TAU} R={R} u0={U0})"]
    for step in range(0, STEPS + 1, EVERY):
        if step:
            lat.step(EVERY)
        F = lat.diagnostics()["force_on_solid"]
        lines.append(f"{step} {F[0]:.17e} {F[1]:.17e} {F[2]:.17e}")
        print(lines[-1], flush=True)
    with open(os.path.join(HERE, "karman_reduced_forces.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
