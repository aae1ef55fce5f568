"""The next-event (point-detector) estimator on the GPU against the oracle (Sec. 6.3).

Per event the score is w e^{-tau} / (4 pi r^2).  FP64 walk: every event
within 1e-12 relative of the oracle.  FP32 walk: against the oracle's FP32
traversal on the same FP32-rounded inputs (so the pieces are the same and
only the products and sums differ): |d tau| <= 1e-6 (1 + tau) for every
event (each positive term Sigma l is rounded once in FP32), and 1e-5
relative on the events with tau <= 10.  Events inside and outside the mesh, detectors inside and
outside; an event at the detector scores 0; rays that miss the mesh score
the bare inverse square.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from vrc_testutil import mesh32, xs32

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def vrc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1706_07476_amd as vrc_mod
    vrc_mod.load_library()
    return vrc_mod


@pytest.fixture()
def ctx(vrc):
    c = vrc.Context(0)
    yield c
    c.close()


def events(seed, mesh, n, margin=3.0):
    rng = np.random.default_rng(seed)
    lo = mesh.lo - margin
    hi = mesh.lo + mesh.n * mesh.h + margin
    p = rng.uniform(lo, hi, (n, 3))
    e = W.log_uniform_energies(rng, n)
    w = rng.lognormal(0.0, 0.5, n)
    return p, e, w


def gpu_scores(ctx, prec, p, e, w, det, dtype):
    import torch
    dt = torch.float64 if dtype == "f64" else torch.float32
    dev = [torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda:0") for a in (p[:, 0], p[:, 1], p[:, 2], e, w)]
    out = torch.full((p.shape[0],), -1.0, dtype=torch.float64, device="cuda:0")
    ctx.next_event(0, prec, dev[:3], dev[3], dev[4], det, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


DETECTORS = {"inside": (7.3, 9.1, 5.6), "outside": (21.0, -4.5, 8.8)}


@pytest.mark.parametrize("where", ["inside", "outside"])
def test_fp64_walk_matches_oracle(ctx, where):
    mesh = W.slab_mesh(808, 32, 0.5, slab=4)
    xs = W.gen.three_material_xs(809, 2000)
    p, e, w = events(810, mesh, 3000)
    det = DETECTORS[where]
    say(f"case: next-event p64, slab 32^3, 3000 events, detector {where}")
    ctx.set_mesh(0, mesh)
    ctx.set_xs(xs)
    got = gpu_scores(ctx, "p64", p, e, w, det, "f64")
    ref = oracle.next_event(mesh, xs, p[:, 0], p[:, 1], p[:, 2], e, w, det)
    pos = ref > 1e-300
    rel = np.abs(got[pos] - ref[pos]) / ref[pos]
    say(f"  {pos.sum()} positive scores, max rel {rel.max():.3e}")
    assert np.all(got[~pos] <= 1e-300)
    assert rel.max() <= 1e-12


@pytest.mark.parametrize("prec", ["p32_t64", "p32_d64"])
def test_fp32_walk_matches_oracle_on_fp32_inputs(ctx, prec):
    mesh = W.slab_mesh(811, 32, 0.5, slab=4)
    xs = W.gen.three_material_xs(812, 2000)
    p, e, w = events(813, mesh, 3000)
    det = tuple(float(np.float32(v)) for v in DETECTORS["inside"])
    say(f"case: next-event {prec} (FP32 walk), slab 32^3, 3000 events")
    ctx.set_mesh(0, mesh)
    ctx.set_xs(xs)
    got = gpu_scores(ctx, prec, p, e, w, det, "f32")
    m32, x32 = mesh32(mesh), xs32(xs)
    f = lambda a: a.astype(np.float32)
    ref = oracle.next_event(m32, x32, f(p[:, 0]), f(p[:, 1]), f(p[:, 2]), f(e).astype(np.float64),
                            f(w).astype(np.float64), det, precision="f32")
    pos = ref > 1e-300
    # tau of every event from the oracle's score: w e^{-tau} / (4 pi r^2)
    q = np.stack([f(p[:, k]).astype(np.float64) for k in range(3)], axis=1)
    r2 = np.sum((np.asarray(det)[None, :] - q) ** 2, axis=1)
    tau = -np.log(ref[pos] * 4 * math.pi * r2[pos] / f(w).astype(np.float64)[pos])
    dtau = np.abs(np.log(got[pos] / ref[pos]))
    rel = np.abs(got[pos] - ref[pos]) / ref[pos]
    say(f"  {pos.sum()} positive scores: max tau {tau.max():.1f}, max |dtau|/(1+tau) {np.max(dtau / (1 + tau)):.3e}, "
        f"rel error on tau <= 10: {rel[tau <= 10].max():.3e}")
    # Every piece adds Sigma l > 0 rounded once in FP32 (Sigma from the FP32 interpolation of
    # the same rounded table): |dtau| <= ~3 * 2^-24 * tau; bound 1e-6 (1 + tau).
    assert np.all(dtau <= 1e-6 * (1.0 + tau))
    assert rel[tau <= 10].max() <= 1e-5


def test_edge_cases(vrc, ctx):
    import torch
    mesh = W.slab_mesh(814, 16, 1.0, slab=4)
    xs = W.gen.three_material_xs(815, 500)
    ctx.set_mesh(0, mesh)
    ctx.set_xs(xs)
    say("case: next-event edge cases")
    det = (3.5, 4.25, 5.0)
    # an event at the detector, one missing the mesh (both outside, ray parallel to a face, off the mesh)
    p = np.array([[3.5, 4.25, 5.0], [-5.0, -3.0, 2.0], [-5.0, -9.0, 2.0]])
    e = np.array([1e-3, 1e-3, 1e-3])
    w = np.array([2.0, 1.5, 0.5])
    got = gpu_scores(ctx, "p64", p, e, w, (-5.0, 30.0, 2.0), "f64")
    r2 = float(np.sum((np.array([-5.0, 30.0, 2.0]) - p[2]) ** 2))
    assert got[2] == pytest.approx(0.5 / (4 * math.pi * r2), rel=1e-15)   # the segment stays outside the mesh
    got0 = gpu_scores(ctx, "p64", p[:1], e[:1], w[:1], det, "f64")
    assert got0[0] == 0.0
    # no events: nothing to do
    empty = [torch.empty(0, dtype=torch.float64, device="cuda:0") for _ in range(5)]
    ctx.next_event(0, "p64", empty[:3], empty[3], empty[4], det, torch.empty(0, dtype=torch.float64, device="cuda:0"))
    # errors
    with pytest.raises(vrc.VrcError):
        gpu_scores_bad = torch.zeros(1, dtype=torch.float64, device="cuda:0")
        ctx.next_event(5, "p64", [gpu_scores_bad] * 3, gpu_scores_bad, gpu_scores_bad, det, gpu_scores_bad)
    with pytest.raises(vrc.VrcError):
        one = torch.zeros(1, dtype=torch.float64, device="cuda:0")
        ctx.next_event(0, "p64", [one] * 3, one, one, (float("nan"), 0.0, 0.0), one)


@pytest.mark.parametrize("dtype,prec", [("f64", "p64"), ("f32", "p32_t64")])
def test_ordered_path_equals_input_order_path(ctx, dtype, prec):
    """From 65536 events the events are first ordered by estimated path length; every score is the
    same bit for bit as from the events in input order (two calls below the threshold), and a
    sample matches the oracle."""
    import torch
    mesh = W.slab_mesh(816, 48, 0.5, slab=6)
    xs = W.gen.three_material_xs(817, 2000)
    n = 70_001
    p, e, w = events(818, mesh, n, margin=2.0)
    det = (11.3, 12.1, 9.6)
    say(f"case: next-event ordered path {prec}, {n} events, slab 48^3")
    ctx.set_mesh(0, mesh)
    ctx.set_xs(xs)
    dt = torch.float64 if dtype == "f64" else torch.float32
    dev = [torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda:0") for a in (p[:, 0], p[:, 1], p[:, 2], e, w)]
    ordered = torch.full((n,), -1.0, dtype=torch.float64, device="cuda:0")
    ctx.next_event(0, prec, dev[:3], dev[3], dev[4], det, ordered)
    plain = torch.full((n,), -1.0, dtype=torch.float64, device="cuda:0")
    h = n // 2
    ctx.next_event(0, prec, [a[:h] for a in dev[:3]], dev[3][:h], dev[4][:h], det, plain[:h])
    ctx.next_event(0, prec, [a[h:] for a in dev[:3]], dev[3][h:], dev[4][h:], det, plain[h:])
    torch.cuda.synchronize()
    a, b = ordered.cpu().numpy(), plain.cpu().numpy()
    assert np.all(a >= 0.0)
    assert np.array_equal(a, b)
    if dtype == "f64":
        idx = np.arange(0, n, 35)
        ref = oracle.next_event(mesh, xs, p[idx, 0], p[idx, 1], p[idx, 2], e[idx], w[idx], det)
        pos = ref > 1e-300
        rel = np.abs(a[idx][pos] - ref[pos]) / ref[pos]
        say(f"  sample of {idx.size}: max rel vs oracle {rel.max():.3e}")
        assert rel.max() <= 1e-12


@pytest.mark.parametrize("kind", ["rect", "density", "rect+density"])
def test_rectilinear_and_density_meshes(ctx, kind):
    """The walk reads the plane tables on a rectilinear mesh and scales Sigma by the voxel's factor:
    FP64 within 1e-12 per event; the FP32 walk against the oracle's FP32 traversal of the same
    rounded inputs within the bound of the FP32 test above."""
    base = W.rect_mesh(820, (28, 25, 30), lo=(-3.0, 1.0, 0.5), h_min=0.2, h_max=1.1) if "rect" in kind \
        else W.slab_mesh(820, 28, 0.5, slab=4)
    rho = W.density_field(821, base.n_voxels, 0.3, 2.5, frac_zero=0.05) if "density" in kind else None
    mesh = W.RectMesh(base.planes, base.mat, rho) if "rect" in kind else W.Mesh(base.lo, base.h, base.n, base.mat, rho)
    xs = W.gen.three_material_xs(822, 2000)
    hi = mesh.hi if "rect" in kind else mesh.lo + mesh.n * mesh.h
    rng = np.random.default_rng(823)
    n = 3000
    p = rng.uniform(mesh.lo - 2.0, hi + 2.0, (n, 3))
    e = W.log_uniform_energies(rng, n)
    w = rng.lognormal(0.0, 0.5, n)
    det = tuple(float(v) for v in (0.5 * (mesh.lo + hi) + np.array([0.137, -0.211, 0.173])))
    say(f"case: next-event on a {kind} mesh, {n} events")
    ctx.set_mesh(0, mesh)
    ctx.set_xs(xs)
    got = gpu_scores(ctx, "p64", p, e, w, det, "f64")
    ref = oracle.next_event(mesh, xs, p[:, 0], p[:, 1], p[:, 2], e, w, det)
    pos = ref > 1e-300
    rel = np.abs(got[pos] - ref[pos]) / ref[pos]
    say(f"  FP64: {pos.sum()} positive scores, max rel {rel.max():.3e}")
    assert np.all(got[~pos] <= 1e-300)
    assert rel.max() <= 1e-12
    # FP32 walk (p32_t64) on the FP32-rounded inputs
    det32 = tuple(float(np.float32(v)) for v in det)
    got32 = gpu_scores(ctx, "p32_t64", p, e, w, det32, "f32")
    f = lambda a: a.astype(np.float32)
    m32, x32 = mesh32(mesh), xs32(xs)
    ref32 = oracle.next_event(m32, x32, f(p[:, 0]), f(p[:, 1]), f(p[:, 2]), f(e).astype(np.float64),
                              f(w).astype(np.float64), det32, precision="f32")
    pos = ref32 > 1e-300
    q = np.stack([f(p[:, k]).astype(np.float64) for k in range(3)], axis=1)
    r2 = np.sum((np.asarray(det32)[None, :] - q) ** 2, axis=1)
    tau = -np.log(ref32[pos] * 4 * math.pi * r2[pos] / f(w).astype(np.float64)[pos])
    dtau = np.abs(np.log(got32[pos] / ref32[pos]))
    say(f"  FP32: max |dtau|/(1+tau) {np.max(dtau / (1 + tau)):.3e}")
    # each term (rho Sigma) l is rounded twice in FP32 here (the factor's product, then the length's)
    assert np.all(dtau <= 2e-6 * (1.0 + tau))
