"""Gradient fields (Sec. 6) on the GPU: the value field of the Wendland C2 kernel and the four
fields of its transverse kernel -w'/r (particle values c/h^2 and c chi_a/h^2) through the C ABI.

Bars: every field's knots and exact pieces meet the parity bars of the value field (knots and
piece boundaries bit-exact; integer coefficients within 1e-6 of each order's largest value on the
ray, plus one unit, since the two sides project the table independently); the gradient assembled
from the library's pieces equals the one assembled from the oracle's within 1e-6 of the ray's
largest gradient component (the coefficient bar of the order-1 terms carried through the
derivative; measured: about 6e-12); against the analytic gradient it is
within the method's error (8 % of the ray's largest gradient component: the along-ray part is the
derivative of an L2-optimal value approximation).
"""
import numpy as np
import pytest

import synth
from oracle import gradient as G
from tests import gpu_helpers as H

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - needs a GPU
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2401_02896_amd as L  # noqa: E402
from tests.test_gpu_parity import _approx, _check_ray  # noqa: E402

T0, T1 = 0.0, 3.0


def _gpu_pieces(out, r):
    eo = out["exact_offsets"].cpu().numpy()
    et = out["exact_t"][eo[r]:eo[r + 1]].cpu().numpy()
    ee = out["exact_end"][eo[r]:eo[r + 1]].cpu().numpy()
    ec = out["exact_coef"][eo[r]:eo[r + 1]].cpu().numpy()
    return [(int(a), int(b), [int(x) for x in c]) for a, b, c in zip(et, ee, ec)]


def test_gradient_fields_match_oracle():
    xyz, h, val = synth.random_scene(41, 200, h_lo=0.05, h_hi=0.12)
    o, v = synth.random_rays(5, 12)
    scF = H.Scene("wendland", 4, 3, 4096, xyz, h, val, 0.0)
    scG = [H.Scene("wendland_grad", 4, 3, 1024, xyz, h, gv, 0.0) for gv in G.transverse_values(xyz, h, val)]
    outF = _approx(scF, o, v, T0, T1)
    outG = [_approx(s, o, v, T0, T1) for s in scG]
    checked = 0
    for r in range(len(o)):
        fF = scF.oracle_ray(o[r], v[r], T0, T1)
        fG = [s.oracle_ray(o[r], v[r], T0, T1) for s in scG]
        for sc, out, f in [(scF, outF, fF)] + list(zip(scG, outG, fG)):
            assert _check_ray(sc, out, r, f)
        if not fF["pieces"]:
            continue
        lo, hi = fF["pieces"][0][0] * scF.tau, fF["pieces"][-1][1] * scF.tau
        ts = np.random.default_rng(r).uniform(lo, hi, 64)
        ov, vv = o[r].astype(np.float64), v[r].astype(np.float64)
        dF = H.eval_exact_pieces(_gpu_pieces(outF, r), scF.tau, scF.sigma, ts, deriv=True)
        Gs = [H.eval_exact_pieces(_gpu_pieces(out, r), s.tau, s.sigma, ts) for out, s in zip(outG, scG)]
        dF_o = H.eval_exact_pieces(fF["pieces"], scF.tau, scF.sigma, ts, deriv=True)
        Gs_o = [H.eval_exact_pieces(f["pieces"], s.tau, s.sigma, ts) for f, s in zip(fG, scG)]
        grads = np.array([G.gradient(ov + t * vv, xyz, h, val, "wendland") for t in ts])
        for e in np.eye(3):
            got = G.assemble(vv, e, ov, dF, Gs[0], Gs[1:])
            ora = G.assemble(vv, e, ov, dF_o, Gs_o[0], Gs_o[1:])
            ref = grads @ e
            scale = np.max(np.abs(ref))
            assert np.max(np.abs(got - ora)) <= 1e-6 * scale, r
            assert np.max(np.abs(got - ref)) <= 0.08 * scale, (r, e)
        checked += 1
    assert checked >= 8


def _same(a, b):
    assert a.keys() == b.keys()
    for k in a:
        if isinstance(a[k], torch.Tensor):
            assert torch.equal(a[k], b[k]), k
        else:
            assert a[k] == b[k], k


@pytest.mark.parametrize("slots", [None, "0"])
def test_shared_gathering_equals_separate_calls(slots):
    """sph_hoa_approx_rays_shared gives each index exactly what its own sph_hoa_approx_rays call
    gives, with single-pass (per-ray slots) and two-walk gathering, for indices of the same
    particles with other values, kernels, K and D."""
    import os

    xyz, h, val = synth.random_scene(43, 300, h_lo=0.04, h_hi=0.1)
    o, v = synth.random_rays(8, 40)
    gv = G.transverse_values(xyz, h, val)
    scs = [H.Scene("wendland", 4, 3, 4096, xyz, h, val, 1e-3)]
    scs += [H.Scene("wendland_grad", 4, 3, 1024, xyz, h, g, 1e-3) for g in gv]
    scs += [H.Scene("wendland_c4_grad", 3, 2, 64, xyz, h, gv[1], 0.0)]
    idx = [s.index() for s in scs]
    if slots is not None:
        os.environ["SPH_HOA_GATHER_SLOTS"] = slots
    try:
        for exact in (True, False):
            shared = L.sph_hoa_approx_rays_shared(idx, torch.as_tensor(o), torch.as_tensor(v), T0, T1, exact=exact)
            for i, ix in enumerate(idx):
                sep = L.sph_hoa_approx_rays(ix, torch.as_tensor(o), torch.as_tensor(v), T0, T1, exact=exact)
                _same(shared[i], sep)
    finally:
        os.environ.pop("SPH_HOA_GATHER_SLOTS", None)
    assert shared[0]["n_pairs"] > 100


def test_shared_gathering_rejects_other_particles():
    xyz, h, val = synth.random_scene(43, 300, h_lo=0.04, h_hi=0.1)
    a = H.Scene("wendland", 4, 3, 4096, xyz, h, val, 1e-3).index()
    h2 = h.copy()
    h2[17] *= np.float32(1.01)
    b = H.Scene("wendland", 4, 3, 4096, xyz, h2, val, 1e-3).index()
    o, v = synth.random_rays(8, 4)
    with pytest.raises(RuntimeError, match="E_INVALID_ARG"):
        L.sph_hoa_approx_rays_shared([a, b], torch.as_tensor(o), torch.as_tensor(v), T0, T1)
    # empty ray set: nothing to gather, every field empty
    out = L.sph_hoa_approx_rays_shared([a, a], torch.zeros((0, 3)), torch.zeros((0, 3)), T0, T1)
    assert [x["n_pieces"] for x in out] == [0, 0]
    # one index several times (with timing on: a sharing call records no gathering time): every
    # field equals the single call
    a.set_timing(True)
    outs = L.sph_hoa_approx_rays_shared([a, a, a], torch.as_tensor(o), torch.as_tensor(v), T0, T1)
    st = a.stats()
    assert st["n_rays"] == len(o)
    ref = L.sph_hoa_approx_rays(a, torch.as_tensor(o), torch.as_tensor(v), T0, T1)
    for x in outs:
        _same(x, ref)


def test_full_size_gradient_fields_sampled():
    """The gradient workload at full size (the plain frame's 1M clustered particles and 512 x 512
    pixel-centre rays, K = 4, D = 3, tol 1e-3): the five fields of one shared call over all rays,
    the benchmark's launch configuration, equal five separate calls bit for bit, and the exact
    pieces of sampled rays meet the parity bars against the oracle."""
    from oracle import geometry

    xyz, h, val = synth.clustered_particles()
    scs = [H.Scene("wendland", 4, 3, 4096, xyz, h, val, 1e-3)]
    scs += [H.Scene("wendland_grad", 4, 3, 4096, xyz, h, g, 1e-3) for g in G.transverse_values(xyz, h, val)]
    idx = [s.index() for s in scs]
    oo, vv = geometry.camera_rays(synth.plain_camera())
    o32 = torch.as_tensor(oo.astype(np.float32))
    v32 = torch.as_tensor(vv.astype(np.float32))
    shared = L.sph_hoa_approx_rays_shared(idx, o32, v32, 1.0, 3.0)
    assert shared[0]["n_pairs"] > 1.5e8
    for i, ix in enumerate(idx):
        sep = L.sph_hoa_approx_rays(ix, o32, v32, 1.0, 3.0)
        _same(shared[i], sep)
        del sep
    del shared
    pix = np.array([512 * 256 + 256, int(np.random.default_rng(78).integers(0, 512 * 512))])
    out = L.sph_hoa_approx_rays_shared(idx, o32[pix], v32[pix], 1.0, 3.0, exact=True)
    for k, r in enumerate(pix):
        for sc, o in zip(scs, out):
            f = sc.oracle_ray(o32[r].numpy(), v32[r].numpy(), 1.0, 3.0)
            _check_ray(sc, o, k, f)
