"""Float accumulation variant (sph_hoa_float_rays, Sec. 4.1) against the oracle's float32 sweep.

Both sides are handed the same float64 table (the oracle's knots and projection jumps, through
sph_hoa_params.knot_table / jump_table), so that every float32 input is the same rounding of the
same value; hit sets, closest points and table entries are bit-identical to the exact path's, and
the sweep's float32 operations are specified one by one.  The pieces must therefore be identical,
bit for bit, with and without reinitialization knots.
"""
import numpy as np
import pytest

import synth
from oracle import floatpath as fp
from oracle import lut
from tests.golden.make_knot_tables import load as load_knots

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - needs a GPU
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2401_02896_amd as L  # noqa: E402

KIND_ID = {"cubic": L.KERNEL_CUBIC, "wendland": L.KERNEL_WENDLAND_C2}
_TABLES = {}


def _table(kind, K, D, n):
    key = (kind, K, D, n)
    if key not in _TABLES:
        theta = load_knots(kind, K, D, n)
        lams = lut.lambda_midpoints(kind, n)
        P = (K + 1) // 2
        shat = np.zeros((n, P, D + 1))
        smid = np.zeros((n, D + 1))
        for i in range(n):
            shat[i], smid[i] = lut.difference_coefficients(kind, float(lams[i]), theta[i], K, D)
        _TABLES[key] = {"theta": theta, "shat": shat, "smid": smid}
    return _TABLES[key]


def _index(kind, K, D, n, xyz, h, val):
    t = _table(kind, K, D, n)
    return L.sph_hoa_build_index(xyz, h, val, kernel=KIND_ID[kind], degree=D, pieces=K, lut_entries=n,
                                 knot_table=t["theta"], jump_table=t["shat"],
                                 jump_table_mid=t["smid"] if K % 2 == 0 else None), t


def _compare(out, r, ref, D):
    o = int(out["ray_offsets"][r])
    c = int(out["ray_counts"][r])
    assert c == len(ref), (r, c, len(ref))
    if c == 0:
        return
    t0 = out["t_start"][o:o + c].cpu().numpy()
    t1 = out["t_end"][o:o + c].cpu().numpy()
    cf = out["coef"][o:o + c].cpu().numpy()
    assert np.array_equal(t0, np.array([p[0] for p in ref], np.float32)), r
    assert np.array_equal(t1, np.array([p[1] for p in ref], np.float32)), r
    assert np.array_equal(cf, np.array([p[2] for p in ref], np.float32)), r


@pytest.mark.parametrize("spec", [("wendland", 2, 2, 256), ("cubic", 3, 3, 256), ("wendland", 4, 1, 256)])
@pytest.mark.parametrize("n_reinit", [0, 7])
def test_float_sweep_bit_identical_to_oracle(spec, n_reinit):
    kind, K, D, n = spec
    xyz, h, val = synth.tiny_particles()
    idx, tab = _index(kind, K, D, n, xyz, h, val)
    o, v = synth.ortho_rays()
    out = L.sph_hoa_float_rays(idx, o, v, 0.0, 1.4, n_reinit=n_reinit)
    assert out["n_pairs"] > 100000
    rng = np.random.default_rng(5)
    for r in np.concatenate([[0, 63, 4095], rng.integers(0, 4096, 9)]):
        ref = fp.ray_pieces(o[r], v[r], 0.0, 1.4, xyz, h, val, tab, K, D, kind, n_reinit=n_reinit)
        _compare(out, int(r), ref, D)
    idx.free()


def test_heavy_rays_through_a_cluster():
    """Rays through a cluster core (hundreds of hits each, several work-group passes of the knot
    loops), next to rays that miss everything."""
    kind, K, D, n = "wendland", 2, 2, 256
    xyz, h, val = synth.clustered_particles(seed=7, n=300_000, clusters=1)
    idx, tab = _index(kind, K, D, n, xyz, h, val)
    rng = np.random.default_rng(11)
    o = np.tile(np.array([[0.5, 0.5, -1.0]], np.float32), (6, 1))
    tgt = np.array([0.5, 0.5, 0.5]) + rng.normal(0, 0.01, (6, 3))
    tgt[5] = [5.0, 5.0, 0.5]  # misses the cube
    v = (tgt - o) / np.linalg.norm(tgt - o, axis=1, keepdims=True)
    v = v.astype(np.float32)
    for n_reinit in (0, 10):
        out = L.sph_hoa_float_rays(idx, o, v, 0.5, 3.0, n_reinit=n_reinit)
        assert int(out["ray_offsets"][1] - out["ray_offsets"][0]) > 3 * 256  # > 256 hits on ray 0
        for r in range(6):
            ref = fp.ray_pieces(o[r], v[r], 0.5, 3.0, xyz, h, val, tab, K, D, kind, n_reinit=n_reinit)
            _compare(out, r, ref, D)
    idx.free()


def test_empty_and_errors():
    xyz, h, val = synth.tiny_particles()
    idx, _ = _index("wendland", 2, 2, 256, xyz, h, val)
    out = L.sph_hoa_float_rays(idx, np.zeros((0, 3), np.float32), np.zeros((0, 3), np.float32), 0.0, 1.0)
    assert out["n_pairs"] == 0
    o, v = synth.ortho_rays(4, 4)
    with pytest.raises(L.SphHoaError):
        L.sph_hoa_float_rays(idx, o, v, 0.0, 1.4, n_reinit=5000)
    with pytest.raises(L.SphHoaError):
        L.sph_hoa_float_rays(idx, o, v, 1.0, 0.5)
    idx.free()
