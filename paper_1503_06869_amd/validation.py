"""The paper's single-particle validations (Sec. 5.1 setup and its appendix
table) -- a spherocylinder rotating under a constant torque, and one
sedimenting under a constant force in a box closed by free-slip walls --
and the tumbling pair of Sec. 6.

    python -m paper_1503_06869_amd.validation [--aspect 4] [--n 816] [--steps 40000]
    python -m paper_1503_06869_amd.validation --case tumbling [--aspect 12] [--dist 14.8] [--n 576]
    python -m paper_1503_06869_amd.validation --case sedimentation [--aspect 8]
        [--orientation lengthwise|sidewise] [--nxy 160] [--nz 1200] [--steps 80000]

The paper's setup: spherocylinders of radius r = 4 dx and L = (1/eps) r
(L including the caps), dx = 1e-5 m, water (nu = 1e-6 m^2/s, rho_f =
1e3 kg/m^3), tau = 6 (so dt = (tau - 1/2)/3 dx^2 / nu), particle density
1195 kg/m^3, a constant torque perpendicular to the axis from its table of
torques, the particle at the centre of an 816^3 cube.  The run reports the
terminal angular velocity next to the paper's LBM value omega*_LBM and the
Tirado value omega_Tir,wC (Eq. CapsTheorRotatMotionTirado for a cylinder of
the full length, with the end correction of Eq. EndeffCorrRotatMotionTirado).

With --all-walls the cube has resting no-slip walls on all six faces, as in
the paper; without, at the z ends only, periodic in x and y.
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


def run(aspect, n, steps, every, log=print, walls=False):
    """walls: resting no-slip walls on all six faces (the paper's cube);
    otherwise on the z faces only, periodic in x and y."""
    from . import lbm
    L = aspect * R_CELLS
    m_lat = lattice_torque(TORQUE[aspect] * 1e-15)
    g = lbm.Context(n, n, n, tau=TAU, wall_u=0.0, init_couette=False, x_walls=walls, y_walls=walls)
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
        "aspect": aspect, "n": n, "steps": steps, "walls": "all six faces" if walls else "z faces",
        "length_cells": L, "radius_cells": R_CELLS,
        "tau": TAU, "dt_s": dt(), "torque_lattice": m_lat,
        "omega_lattice": w_lat, "omega_per_s": w,
        "omega_spread_pct": float(100.0 * (tail.max() - tail.min()) / abs(w_lat)) if w_lat else None,
        "omega_paper_lbm": OMEGA_LBM[aspect],
        "omega_tirado_wc": tirado_rotation(TORQUE[aspect] * 1e-15, L * DX, R_CELLS * DX),
        "dev_vs_paper_lbm_pct": 100.0 * (w / OMEGA_LBM[aspect] - 1.0),
        "history": list(zip(ts, ws)),
    }


# ---------------------------------------------------------------------------
# Two tumbling, sedimenting spherocylinders (Sec. 6 setup and results): r = 4
# dx with dx = 4.98e-6 m, L = (1/eps) r, water, tau = 6, particle density
# 1492 kg/m^3, side by side in x at centre distance dist, axes along the
# force (z), in a fully periodic cube with momentum stabilization, pushed
# along z by the buoyancy-corrected weight of its table of forces.
TUMBLE_DX = 4.98e-6      # m
TUMBLE_RHO_P = 1492.0    # kg/m^3
TUMBLE_FORCE = {10: 1.119e-9, 12: 1.358e-9, 14: 1.598e-9}   # F_z [kg m/s^2]
# first tumbling period in the 576^3 box (its table of the time evolution):
# (aspect, dist [dx]) -> D* [m], T* [s], U* [m/s]
TUMBLE_PERIOD1 = {(10, 16.0): (4.38e-3, 2.71, 1.61e-3), (12, 14.8): (4.18e-3, 2.13, 1.96e-3)}


def tumble_dt():
    """nu = (tau - 1/2)/3 dx^2/dt (Eq. kinVisc) at the tumbling dx."""
    return (TAU - 0.5) / 3.0 * TUMBLE_DX * TUMBLE_DX / NU


def lattice_force(force_si, dx=None, dt_s=None):
    """kg m/s^2 to lattice units (mass rho_f dx^3, length dx, time dt)."""
    dx = TUMBLE_DX if dx is None else dx
    dt_s = tumble_dt() if dt_s is None else dt_s
    return force_si / (RHO_F * dx ** 4 / dt_s ** 2)


def tumbling_periods(steps, axis_xz, z):
    """Tumbling periods of one particle from samples of its axis (t_x, t_z)
    and its unwrapped z position: a period ends each time the axis has turned
    by another half revolution from its start (the shape is symmetric under
    t -> -t, so the doubled angle is used).  Crossings are interpolated
    linearly between samples.  Returns [(step_end, z_end)] for the period
    ends, the start (0, z[0]) first."""
    t = np.asarray(axis_xz, dtype=np.float64)
    phi = np.unwrap(np.arctan2(2.0 * t[:, 0] * t[:, 1], t[:, 1] ** 2 - t[:, 0] ** 2))
    turn = np.abs(phi - phi[0]) / (2.0 * np.pi)
    ends = [(float(steps[0]), float(z[0]))]
    k = 1
    for i in range(1, len(turn)):
        while turn[i - 1] < k <= turn[i]:
            w = (k - turn[i - 1]) / (turn[i] - turn[i - 1])
            ends.append((steps[i - 1] + w * (steps[i] - steps[i - 1]), z[i - 1] + w * (z[i] - z[i - 1])))
            k += 1
    return ends


def run_tumbling(aspect, n, dist, steps, every, storage="f32", contact_k=0.0, contact_range=2.0, log=print):
    """contact_k, contact_range: the short-range repulsion standing in for the
    paper's collision handling (off at 0); the trailing ends of the pair
    approach each other within the first tenth of a revolution."""
    from . import lbm
    L = aspect * R_CELLS
    F = lattice_force(TUMBLE_FORCE[aspect])
    g = lbm.Context(n, n, n, tau=TAU, z_periodic=True, stabilize=True, storage=storage, contact_k=contact_k,
                    contact_range=contact_range)
    c = 0.5 * (n - 1)
    q = (math.cos(math.pi / 4), 0.0, -math.sin(math.pi / 4), 0.0)   # axis along +z
    for s in (-1.0, 1.0):
        g.add_fiber((c + 0.5 * s * dist, c, c), q, L, R_CELLS, TUMBLE_RHO_P / RHO_F, shape="spherocylinder",
                    force=(0.0, 0.0, F))
    rows = []
    zu, zprev = None, None
    t0 = time.time()
    done = 0
    while done < steps:
        k = min(every, steps - done)
        g.step(k)
        done += k
        X, qq, V, W = g.fiber_state()
        t = np.array([1.0 - 2.0 * (qq[0, 2] ** 2 + qq[0, 3] ** 2), 2.0 * (qq[0, 1] * qq[0, 2] + qq[0, 0] * qq[0, 3]),
                      2.0 * (qq[0, 1] * qq[0, 3] - qq[0, 0] * qq[0, 2])])
        z = X[0, 2]
        if zu is None:
            zu = z
        else:
            dz = z - zprev
            zu += dz - n * round(dz / n)
        zprev = z
        sep = (X[1, 0] - X[0, 0]) % n
        rows.append([done, t[0], t[2], zu, V[0, 0], V[0, 2], sep])
        if done % (10 * every) == 0 or done == steps:
            log("step %7d  axis (%.3f, %.3f)  z %.2f  V (%.3e, %.3e)  sep %.2f  %.0f s"
                % (done, t[0], t[2], zu, V[0, 0], V[0, 2], sep, time.time() - t0))
    g.close()
    h = np.asarray(rows)
    ends = tumbling_periods(np.r_[0.0, h[:, 0]], np.r_[[[0.0, 1.0]], h[:, 1:3]],
                            np.r_[c, h[:, 3]])
    dts = tumble_dt()
    periods = []
    for (s0, z0), (s1, z1) in zip(ends[:-1], ends[1:]):
        sel = (h[:, 0] >= s0) & (h[:, 0] <= s1)
        T = (s1 - s0) * dts
        D = (z1 - z0) * TUMBLE_DX
        periods.append({"T_s": T, "D_m": D, "U_m_s": D / T,
                        "ux_min_m_s": float(h[sel, 4].min() * TUMBLE_DX / dts),
                        "ux_max_m_s": float(h[sel, 4].max() * TUMBLE_DX / dts),
                        "uz_min_m_s": float(h[sel, 5].min() * TUMBLE_DX / dts),
                        "uz_max_m_s": float(h[sel, 5].max() * TUMBLE_DX / dts),
                        "sep_min_dx": float(h[sel, 6].min()), "sep_max_dx": float(h[sel, 6].max())})
    ref = TUMBLE_PERIOD1.get((aspect, float(dist)))
    return {"aspect": aspect, "n": n, "dist_dx": dist, "steps": steps, "storage": storage,
            "contact_k": contact_k, "contact_range": contact_range,
            "dt_s": dts, "force_lattice": F, "periods": periods,
            "paper_period1": {"D_m": ref[0], "T_s": ref[1], "U_m_s": ref[2]} if ref else None,
            "history": h.tolist()}


# ---------------------------------------------------------------------------
# Translational validation (Sec. 5.1 setup): the same spherocylinders under
# the constant force F_z = 5.128e-10 N (the buoyancy-corrected weight of a
# sphere of radius 4 dx) in a cuboid closed by free-slip walls, the particle
# centred in x and y and 100 r below the top wall (z = 0), falling towards
# +z.  The appendix table's LBM velocities U*_LBM [1e-6 m/s] (2560^2 x 2688
# box) and the Tirado values for a cylinder of the full length (wC) and of
# the length without the caps (nC), by orientation of the axis relative to
# the force.
SED_FORCE = 5.128e-10    # kg m/s^2
U_LBM = {"lengthwise": {4: 503, 6: 419, 8: 363, 10: 324, 12: 294, 14: 269},
         "sidewise": {4: 447, 6: 349, 8: 291, 10: 252, 12: 223, 14: 201}}
U_TIR_WC = {"lengthwise": {4: 481, 6: 409, 8: 361, 10: 325, 12: 297, 14: 273},
            "sidewise": {4: 429, 6: 344, 8: 292, 10: 255, 12: 227, 14: 205}}


def tirado_translation(force, length, radius, orientation, mu=RHO_F * NU):
    """Sedimentation velocity F / gamma_t of a cylinder (Eqs.
    CapsTheorVelLengthwSidesMotionTirado, EndeffLengthwMotionTirado,
    EndeffCorrSidewMotionTirado): gamma_par = 2 pi mu L / (ln a + v_par),
    gamma_perp = 4 pi mu L / (ln a + v_perp), a = L / (2 r),
    v_par = -0.207 + 0.980/a - 0.133/a^2, v_perp = 0.839 + 0.185/a + 0.233/a^2."""
    a = length / (2.0 * radius)
    if orientation == "lengthwise":
        gamma = 2.0 * math.pi * mu * length / (math.log(a) - 0.207 + 0.980 / a - 0.133 / a ** 2)
    else:
        gamma = 4.0 * math.pi * mu * length / (math.log(a) + 0.839 + 0.185 / a + 0.233 / a ** 2)
    return force / gamma


def run_sedimentation(aspect, orientation, nxy, nz, steps, every=200, storage="f32", window=0.34, log=print):
    """One spherocylinder sedimenting in a free-slip nxy x nxy x nz box.
    The terminal velocity is the mean of the samples (every `every` steps)
    in the last `window` of the run, as the paper averages its samples."""
    from . import lbm
    L = aspect * R_CELLS
    F = lattice_force(SED_FORCE, DX, dt())
    g = lbm.Context(nxy, nxy, nz, tau=TAU, storage=storage, x_walls="free-slip", y_walls="free-slip",
                    z_free_slip=True)
    c = 0.5 * (nxy - 1)
    z0 = 100.0 * R_CELLS - 0.5            # the top wall lies half a cell above cell 0
    axis = (0.0, 0.0, 1.0) if orientation == "lengthwise" else (1.0, 0.0, 0.0)
    t = np.asarray(axis)
    q = np.array([1.0 + t[0], 0.0, -t[2], t[1]])
    q = q / np.linalg.norm(q)
    g.add_fiber((c, c, z0), q, L, R_CELLS, RHO_P / RHO_F, shape="spherocylinder", force=(0.0, 0.0, F))
    ts, us, zs = [], [], []
    t0 = time.time()
    done = 0
    while done < steps:
        k = min(every, steps - done)
        g.step(k)
        done += k
        X, _, V, _ = g.fiber_state()
        ts.append(done)
        us.append(float(V[0][2]))
        zs.append(float(X[0][2]))
        if len(ts) % max(1, 5000 // every) == 0 or done == steps:
            log("step %7d  U_z %.6e (lattice)  %.2f um/s  z %.1f  %.0f s" % (
                done, us[-1], us[-1] * DX / dt() * 1e6, zs[-1], time.time() - t0))
    g.close()
    tail = np.asarray(us[int(len(us) * (1.0 - window)):])
    u_lat = float(tail.mean())
    u = u_lat * DX / dt()
    return {
        "aspect": aspect, "orientation": orientation, "nxy": nxy, "nz": nz, "steps": steps,
        "storage": storage, "walls": "free-slip on all six faces",
        "length_cells": L, "radius_cells": R_CELLS, "tau": TAU, "dt_s": dt(), "force_lattice": F,
        "u_lattice": u_lat, "u_m_s": u,
        "delta_u_pct": float(100.0 * (tail.max() - tail.min()) / abs(u_lat)) if u_lat else None,
        "re_p_d": u * 2.0 * R_CELLS * DX / NU,
        "z_end": zs[-1],
        "u_paper_lbm_2560": U_LBM[orientation][aspect] * 1e-6,
        "u_tirado_wc": tirado_translation(SED_FORCE, L * DX, R_CELLS * DX, orientation),
        "history": list(zip(ts, us, zs)),
    }


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--case", default="rotation", choices=("rotation", "tumbling", "sedimentation"))
    ap.add_argument("--orientation", default="lengthwise", choices=("lengthwise", "sidewise"))
    ap.add_argument("--nxy", type=int, default=160)
    ap.add_argument("--nz", type=int, default=1200)
    ap.add_argument("--aspect", type=int, default=None)
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--dist", type=float, default=14.8)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--every", type=int, default=None)
    ap.add_argument("--storage", default="f32")
    ap.add_argument("--contact-k", type=float, default=0.0)
    ap.add_argument("--contact-range", type=float, default=2.0)
    ap.add_argument("--all-walls", action="store_true", help="rotation: no-slip walls on all six faces")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    if a.case == "sedimentation":
        res = run_sedimentation(a.aspect or 8, a.orientation, a.nxy, a.nz, a.steps or 80000, a.every or 200,
                                a.storage, log=lambda s: print(s, flush=True))
        line = {k: v for k, v in res.items() if k != "history"}
        print(json.dumps(line), flush=True)
        if a.out:
            with open(a.out, "w") as fh:
                json.dump(res, fh)
        return 0
    if a.case == "tumbling":
        res = run_tumbling(a.aspect or 12, a.n or 576, a.dist, a.steps or 50000, a.every or 200, a.storage,
                           a.contact_k, a.contact_range, log=lambda s: print(s, flush=True))
        line = {k: v for k, v in res.items() if k != "history"}
        print(json.dumps(line), flush=True)
        if a.out:
            with open(a.out, "w") as fh:
                json.dump(res, fh)
        return 0
    res = run(a.aspect or 4, a.n or 816, a.steps or 40000, a.every or 1000, log=lambda s: print(s, flush=True),
              walls=a.all_walls)
    line = {k: v for k, v in res.items() if k != "history"}
    print(json.dumps(line), flush=True)
    if a.out:
        with open(a.out, "w") as fh:
            json.dump(res, fh)
    return 0


if __name__ == "__main__":
    sys.exit(main())
