"""Pins of how the oracle composes its independently pinned pieces.

Docking: a restart is its placement followed by S sweeps, each sweep the
rotation scans about x, y, z, the translation scans along x, y, z and the
torsion scans of bonds 0..K-1 in the given order; the trace and the per-scan
best scores follow that order slot by slot, and the final score is the
trilinear score of the last pose.  The test below rebuilds every restart of
``oracle.dock_ligand`` from ``oracle.place`` and single ``oracle.scan`` calls
(each pinned on its own in test_oracle_pins.py) and requires identical bits,
for S = 1..3, K = 0 and K > 0, in FP32 and FP64.  A swapped scan order or an
off-by-one sweep count changes poses and traces, which the negative control
shows for these inputs.

Refinement: the step rule (step sizes, the norm clip of the translation and
rotation blocks, the per-bond clip of the torsion steps, and the halving of
the step scale after a rejected step) is pinned by closed forms on a linear
grid, where every atom's trilinear gradient is (alpha/h, 0, 0):
  * a two-atom rod off the pivot turns about -z by
    min(eta_w * |torque|, clip_w) per step, |torque| = (alpha/h) * sum_i d_i cos(theta),
    while it moves +x by min(eta_t * 2 alpha/h, clip_t);
  * one moving atom at angle phi about a bond axis along +z turns by
    clamp(-eta_th * (alpha/h) * rho * sin(phi), +-clip_th);
  * with a static atom placed so that a full clipped torsion step clashes and
    shorter ones do not, the steps alternate rejected / accepted and the
    accepted angle after 2n steps is phi0 - clip (1 - 2^-n).
"""
import numpy as np
import pytest

import gen
import oracle
from test_oracle_pins import make_pocket

def rebuild_restart(lig, pk, row, angles, T, S, bits):
    """Placement, then S x [rot x,y,z; trans x,y,z; torsions 0..K-1], from single scans."""
    fp64 = bits == 64
    xyz, P = oracle.place(lig, row, pk.center.astype(np.float64), bits=bits, fp64_input=fp64)
    trace, best = [], []
    for _ in range(S):
        order = [(0, e) for e in range(3)] + [(1, e) for e in range(3)] + [(2, k) for k in range(lig["K"])]
        row_t, row_b = [], []
        for kind, which in order:
            j, xyz, P, _, _, b = oracle.scan(lig, pk, angles, T, oracle.trans_step(T), oracle.CLASH2, kind, which,
                                             xyz, P, bits=bits, fp64_input=fp64)
            row_t.append(j)
            row_b.append(b)
        trace.append(row_t)
        best.append(row_b)
    return xyz, P, np.array(trace, np.int64).reshape(S, 6 + lig["K"]), np.array(best).reshape(S, 6 + lig["K"])


def composition_cases(tiny):
    L = tiny["ligs"]
    rigid = gen.ligands_from_sizes(np.array([777]), 4, np.array([23]), np.array([0]))
    return [L.ligand(0), L.ligand(5), L.ligand(11), rigid.ligand(0)]


@pytest.mark.parametrize("bits", [32, 64])
@pytest.mark.parametrize("S", [1, 2, 3])
def test_restart_is_placement_then_sweeps_in_order(tiny, bits, S):
    pk = tiny["pocket"]
    rows = [0, 3, 7]
    rt = (tiny["r32"] if bits == 32 else tiny["r64"]).astype(np.float64)[rows]
    at = (tiny["a32"] if bits == 32 else tiny["a64"]).astype(np.float64)
    T = tiny["w"].angle_samples
    cases = composition_cases(tiny)
    assert cases[-1]["K"] == 0 and all(c["K"] > 0 for c in cases[:-1])
    for lig in cases:
        d = oracle.dock_ligand(lig, pk, rt, at, T, S, oracle.trans_step(T), oracle.CLASH2, bits=bits,
                               fp64_input=bits == 64, want_scan_scores=True)
        assert d["trace"].shape == (len(rows), S, 6 + lig["K"])
        for r, row in enumerate(rt):
            xyz, P, tr, best = rebuild_restart(lig, pk, row, at, T, S, bits)
            np.testing.assert_array_equal(d["trace"][r], tr, err_msg=f"N={lig['N']} K={lig['K']} restart {r} trace")
            np.testing.assert_array_equal(d["scan_scores"][r], best)
            np.testing.assert_array_equal(d["poses"][r], xyz)
            np.testing.assert_array_equal(d["pivots"][r], P)
            assert d["final"][r] == oracle.score(pk, xyz, 1, bits)


def test_composition_is_sensitive_to_order_and_sweep_count(tiny):
    """Negative control: translations before rotations, or one sweep fewer, give
    other poses on these inputs, so the equality above is not vacuous."""
    pk = tiny["pocket"]
    rt = tiny["r32"].astype(np.float64)[[0, 3, 7]]
    at = tiny["a32"].astype(np.float64)
    T = tiny["w"].angle_samples
    differ_order = differ_count = 0
    for lig in composition_cases(tiny)[:3]:
        d = oracle.dock_ligand(lig, pk, rt, at, T, 2, oracle.trans_step(T), oracle.CLASH2, bits=32)
        d1 = oracle.dock_ligand(lig, pk, rt, at, T, 1, oracle.trans_step(T), oracle.CLASH2, bits=32)
        for r, row in enumerate(rt):
            xyz, P = oracle.place(lig, row, pk.center.astype(np.float64), bits=32)
            for _ in range(2):
                for kind, which in [(1, e) for e in range(3)] + [(0, e) for e in range(3)] + \
                        [(2, k) for k in range(lig["K"])]:
                    _, xyz, P, _, _, _ = oracle.scan(lig, pk, at, T, oracle.trans_step(T), oracle.CLASH2, kind,
                                                     which, xyz, P, bits=32)
            differ_order += not np.array_equal(xyz, d["poses"][r])
            differ_count += not np.array_equal(d1["poses"][r], d["poses"][r])
    assert differ_order > 0 and differ_count > 0


# ---------------------------------------------------------------- refinement step rule
# distinct rates and clips, so that a step that took another block's rate or clip fails
ETA = dict(eta_t=1e-2, eta_w=1.5e-3, eta_th=0.7e-3, clip_t=0.1, clip_w=0.05, clip_th=0.1)


def linear_pocket(alpha):
    """Grid value alpha * ix on a 64^3 grid at h = 0.5 from -16 A: the trilinear
    gradient is (alpha / h, 0, 0) everywhere inside."""
    n = 64
    ix = np.broadcast_to(np.arange(n, dtype=np.float64), (n, n, n))
    return make_pocket((alpha * ix).astype(np.float32), origin=(-16.0, -16.0, -16.0), h=0.5)


def custom_ligand(xyz, frag_mask, bonds):
    xyz = np.asarray(xyz, np.float64)
    N, K = len(xyz), len(bonds)
    ta = np.array([b[0] for b in bonds], np.int32)
    tb = np.array([b[1] for b in bonds], np.int32)
    inv = np.array([1.0 / np.linalg.norm(xyz[b] - xyz[a]) for a, b in bonds], np.float64)
    c = xyz.mean(0)
    return dict(N=N, K=K, xyz=xyz, xyz64=xyz, parent=np.full(N, -1, np.int32),
                frag_mask=np.asarray(frag_mask, np.uint32), tors_a=ta, tors_b=tb, inv_len=inv, inv_len64=inv,
                ref=c, ref64=c)


@pytest.mark.parametrize("alpha", [2.0, 20.0])   # rotation step below / above its clip
def test_refine_rigid_rotation_step_rod(alpha):
    h = 0.5
    G = alpha / h
    P = np.array([0.3, -0.2, 0.1])
    d = np.array([1.0, 2.5])                  # distances of the two atoms from the pivot, along +y
    lig = custom_ligand(P + np.outer(d, [0.0, 1.0, 0.0]), [0, 0], [])
    pk = linear_pocket(alpha)
    steps = 20
    s, out, acc = oracle.refine(lig, pk, lig["xyz"], P, bits=64, fp64_input=True, steps=steps, **ETA)
    assert acc == steps
    theta, t = 0.0, 0.0
    clipped = 0
    for _ in range(steps):
        torque = G * d.sum() * np.cos(theta)          # along -z
        dth = min(ETA["eta_w"] * torque, ETA["clip_w"])
        clipped += dth == ETA["clip_w"]
        theta += dth
        t += min(ETA["eta_t"] * 2 * G, ETA["clip_t"])
    expect = P + np.stack([t + d * np.sin(theta), d * np.cos(theta), np.zeros(2)], 1)
    np.testing.assert_allclose(out, expect, rtol=0, atol=1e-9)
    assert (clipped == 0) == (alpha == 2.0) and (clipped > 0) == (alpha == 20.0)
    assert s == pytest.approx(alpha * ((out[:, 0] + 16.0) / h).sum(), abs=1e-8)


def torsion_chain(phi0, rho=1.4, zm=2.0, static=(-1.2, -0.9, -0.6)):
    """Atom 0 = bond pivot a at the origin, atom 1 = b on +z, atom 2 moves with the
    bond on a circle of radius rho at height zm, atom 3 static."""
    xyz = [[0.0, 0.0, 0.0], [0.0, 0.0, 1.5], [rho * np.cos(phi0), rho * np.sin(phi0), zm], list(static)]
    return custom_ligand(xyz, [0, 1, 1, 0], [(0, 1)])


@pytest.mark.parametrize("alpha", [2.0, 100.0])   # torsion step below / above its clip
def test_refine_torsion_step_closed_form(alpha):
    h = 0.5
    G = alpha / h
    rho, phi0 = 1.4, 2.0
    lig = torsion_chain(phi0, rho)
    pk = linear_pocket(alpha)
    prm = dict(ETA, eta_t=0.0, eta_w=0.0)
    steps = 25
    s, out, acc = oracle.refine(lig, pk, lig["xyz"], np.zeros(3), bits=64, fp64_input=True, steps=steps, **prm)
    assert acc == steps
    phi, clipped = phi0, 0
    for _ in range(steps):
        g = -G * rho * np.sin(phi)
        dphi = float(np.clip(prm["eta_th"] * g, -prm["clip_th"], prm["clip_th"]))
        clipped += abs(dphi) == prm["clip_th"]
        phi += dphi
    np.testing.assert_allclose(out[[0, 1, 3]], lig["xyz"][[0, 1, 3]], rtol=0, atol=0)
    np.testing.assert_allclose(out[2], [rho * np.cos(phi), rho * np.sin(phi), 2.0], rtol=0, atol=1e-9)
    assert (clipped == 0) == (alpha == 2.0) and (clipped > 0) == (alpha == 100.0)


def test_refine_rejected_step_halves_the_step_scale():
    """The static atom sits at angle psi on the moving atom's circle; a full
    clipped step (0.1 rad) toward it clashes, 3/4 of it does not.  Steps then
    alternate rejected (scale halved, pose kept) and accepted."""
    rho, phi0, psi, zm = 1.4, 1.0, 0.2, 2.0
    alpha = 100.0
    lig = torsion_chain(phi0, rho, zm, static=(rho * np.cos(psi), rho * np.sin(psi), zm))
    pk = linear_pocket(alpha)
    d2 = lambda phi: 2 * rho * rho * (1 - np.cos(phi - psi))
    clip = ETA["clip_th"]
    # just above a full step's distance: every candidate at phi0 - clip clashes, the
    # accepted angles phi0 - clip (1 - 2^-n), n <= 3, and their half steps do not
    clash2 = d2(phi0 - clip) + 0.1 * (d2(phi0 - 0.75 * clip) - d2(phi0 - clip))
    assert d2(phi0) > clash2
    prm = dict(ETA, eta_t=0.0, eta_w=0.0)
    for steps, accepted in [(1, 0), (2, 1), (3, 1), (4, 2), (6, 3)]:
        s, out, acc = oracle.refine(lig, pk, lig["xyz"], np.zeros(3), bits=64, fp64_input=True, steps=steps,
                                    clash2=clash2, **prm)
        assert acc == accepted, f"{steps} steps"
        phi = phi0 - clip * (1 - 0.5 ** accepted)
        np.testing.assert_allclose(out[2], [rho * np.cos(phi), rho * np.sin(phi), zm], rtol=0, atol=1e-9,
                                   err_msg=f"{steps} steps")
