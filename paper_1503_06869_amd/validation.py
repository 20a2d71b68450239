"""Single-spherocylinder rotation under a constant torque (the paper's
rotational validation, Sec. 5.1 setup and its appendix table).

    python -m paper_1503_06869_amd.validation [--aspect 4] [--n 816] [--steps 40000]

The paper's setup: spherocylinders of radius r = 4 dx and L = (1/eps) r
(L including the caps), dx = 1e-5 m, water (nu = 1e-6 m^2/s, rho_f =
1e3 kg/m^3), tau = 6 (so dt = (tau - 1/2)/3 dx^2 / nu), particle density
1195 kg/m^3, a constant torque perpendicular to the axis from its table of
torques, the particle at the centre of an 816^3 cube.  The run reports the
terminal angular velocity next to the paper's LBM value omega*_LBM and the
Tirado value omega_Tir,wC (Eq. CapsTheorRotatMotionTirado for a cylinder of
the full length, with the end correction of Eq. EndeffCorrRotatMotionTirado).

Difference from the paper's setup: its cube has no-slip walls on all six
faces; this lattice has stationary no-slip walls at the z ends (walls moving
with U = 0) and is periodic in x and y.
"""
import argparse
import json
import math
import sys
import time

import numpy as np

DX = 1e-5            # m
NU = 1e-6            # m^2/s
RHO_F = 1e3          # kg/m^3
RHO_P = 1195.0       # kg/m^3
TAU = 6.0
R_CELLS = 4.0

# Torques M_x [1e-15 kg m^2/s^2] applied for aspect ratios 1/eps (the
# paper's table of torques for the rotational validation) and the angular
# velocities [1/s] of its appendix table: omega*_LBM and omega_Tir,wC.
TORQUE = {4: 12.26, 6: 17.86, 8: 24.62, 10: 32.38, 12: 41.09, 14: 50.68}
OMEGA_LBM = {4: 1.97, 6: 1.18, 8: 0.829, 10: 0.638, 12: 0.519, 14: 0.436}
OMEGA_TIR_WC = {4: 1.36, 6: 0.909, 8: 0.682, 10: 0.545, 12: 0.455, 14: 0.390}


def dt():
    """Time step from nu = (tau - 1/2)/3 dx^2/dt (Eq. kinVisc)."""
    return (TAU - 0.5) / 3.0 * DX * DX / NU


def tirado_rotation(torque, length, radius, mu=RHO_F * NU):
    """Angular velocity M / gamma_r of a cylinder (Eqs. CapsTheorRotatMotionTirado
    and EndeffCorrRotatMotionTirado): gamma_r = pi mu L^3 / (3 (ln a + delta)),
    a = L / (2 r), delta = -0.662 + 0.917/a - 0.050/a^2."""
    a = length / (2.0 * radius)
    delta = -0.662 + 0.917 / a - 0.050 / a ** 2
    gamma = math.pi * mu * length ** 3 / (3.0 * (math.log(a) + delta))
    return torque / gamma


def lattice_torque(torque_si):
    """kg m^2/s^2 to lattice units (mass rho_f dx^3, length dx, time dt)."""
    return torque_si / (RHO_F * DX ** 3 * DX ** 2 / dt() ** 2)


def run(aspect, n, steps, every, log=print):
    from . import lbm
    L = aspect * R_CELLS
    m_lat = lattice_torque(TORQUE[aspect] * 1e-15)
    g = lbm.Context(n, n, n, tau=TAU, wall_u=0.0, init_couette=False)
    c = 0.5 * (n - 1)
    q = (math.cos(math.pi / 4), 0.0, 0.0, math.sin(math.pi / 4))   # axis along y
    g.add_fiber((c, c, c), q, L, R_CELLS, RHO_P / RHO_F, shape="spherocylinder", torque=(m_lat, 0.0, 0.0))
    ts, ws = [], []
    t0 = time.time()
    done = 0
    while done < steps:
        k = min(every, steps - done)
        g.step(k)
        done += k
        _, _, _, W = g.fiber_state()
        ts.append(done)
        ws.append(float(W[0][0]))
        log("step %7d  omega_x %.6e (lattice)  %.4f 1/s  %.0f s" % (done, ws[-1], ws[-1] / dt(),
                                                                     time.time() - t0))
    g.close()
    tail = np.asarray(ws[len(ws) * 3 // 4:])
    w_lat = float(tail.mean())
    w = w_lat / dt()
    return {
        "aspect": aspect, "n": n, "steps": steps, "length_cells": L, "radius_cells": R_CELLS,
        "tau": TAU, "dt_s": dt(), "torque_lattice": m_lat,
        "omega_lattice": w_lat, "omega_per_s": w,
        "omega_spread_pct": float(100.0 * (tail.max() - tail.min()) / abs(w_lat)) if w_lat else None,
        "omega_paper_lbm": OMEGA_LBM[aspect],
        "omega_tirado_wc": tirado_rotation(TORQUE[aspect] * 1e-15, L * DX, R_CELLS * DX),
        "dev_vs_paper_lbm_pct": 100.0 * (w / OMEGA_LBM[aspect] - 1.0),
        "history": list(zip(ts, ws)),
    }


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--aspect", type=int, default=4, choices=sorted(TORQUE))
    ap.add_argument("--n", type=int, default=816)
    ap.add_argument("--steps", type=int, default=40000)
    ap.add_argument("--every", type=int, default=1000)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    res = run(a.aspect, a.n, a.steps, a.every, log=lambda s: print(s, flush=True))
    line = {k: v for k, v in res.items() if k != "history"}
    print(json.dumps(line), flush=True)
    if a.out:
        with open(a.out, "w") as fh:
            json.dump(res, fh)
    return 0


if __name__ == "__main__":
    sys.exit(main())
