"""Pins of the oracle's progressive solver (Sec. 2.2, Eq. 8-9; Algorithm 1)
in a closed furnace: a sphere emitting L_e everywhere with diffuse albedo
rho, whose radiance is L_e / (1 - rho) (the Neumann series L_e + rho L_e +
rho^2 L_e + ... the section writes out)."""
import numpy as np

import oracle
from synth import workloads as W

LE = np.array([1.0, 0.5, 0.25])
RHO = np.array([0.5, 0.6, 0.7])
L_STAR = LE / (1.0 - RHO)


def _run(frames, paths=2048, verts=2):
    o = oracle.Oracle(**W.furnace_table())
    over = -np.inf
    for it in range(frames):
        x, nx, tp, em = W.furnace_paths(paths, verts, it, le=tuple(LE), albedo=tuple(RHO))
        lbar = oracle.progressive_step(o, x, nx, tp, em)
        if it == 0:
            # no cell is blended before the first frame: every sample is L_e
            assert np.all(lbar == LE[:, None])
            assert np.all(o.export()["L"] == LE[:, None])
        over = max(over, float(np.max(o.export()["L"] / L_STAR[:, None] - 1.0)))
    return o, over


def test_first_frame_is_emission_and_values_never_overshoot():
    # every sample is L_e + rho * (a value <= L*) <= L*: no cell passes L*
    _, over = _run(30)
    assert over <= 1e-6


def test_furnace_converges_to_the_closed_form():
    o, _ = _run(200)
    L = o.export()["L"]
    rel = np.abs(L / L_STAR[:, None] - 1.0)
    assert float(np.mean(rel)) < 5e-4
    assert float(np.percentile(rel, 90)) < 1e-3


def test_without_transport_the_solver_keeps_emission():
    """rho = 0: the step transports nothing, every cell stays at L_e."""
    o = oracle.Oracle(**W.furnace_table())
    for it in range(5):
        x, nx, tp, em = W.furnace_paths(512, 2, it, le=tuple(LE), albedo=(0.0, 0.0, 0.0))
        oracle.progressive_step(o, x, nx, tp, em)
    assert np.all(o.export()["L"] == LE[:, None])


def test_radiance_minus_emission_field_of_algorithm_2():
    """Algorithm 2 tracks L_o\\e: the sample at x_i picks the emission of the
    next vertex up through the sampled step instead of its own:
    Lbar = (L_e(x_{i+1}) + L~o\\e(x_{i+1})) t_i, i.e. the step's emission
    argument is t_i L_e.  In the furnace its fixed point is
    L - L_e = rho L_e / (1 - rho)."""
    o = oracle.Oracle(**W.furnace_table())
    for it in range(200):
        x, nx, tp, em = W.furnace_paths(2048, 2, it, le=tuple(LE), albedo=tuple(RHO))
        le_next = tuple(np.float32(r) * e for r, e in zip(RHO, em))
        oracle.progressive_step(o, x, nx, tp, le_next)
    L = o.export()["L"]
    want = (RHO * LE / (1.0 - RHO))[:, None]
    rel = np.abs(L / want - 1.0)
    assert float(np.mean(rel)) < 5e-4 and float(np.percentile(rel, 90)) < 1e-3
