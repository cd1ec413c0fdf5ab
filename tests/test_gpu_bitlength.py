"""Integer bit-length study (Sec. 5.1): the accumulation rule in wrap-around 32/64/96/128-bit
integers on the GPU (sph_hoa_accumulate_bits) against the oracle's exact accumulation reduced
modulo 2^W.  Integer work: every limb must match bit for bit."""
import numpy as np
import pytest

import synth
from oracle import knots

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - needs a GPU
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2401_02896_amd as L  # noqa: E402


def _table(dist, jumps):
    n, dp1, _ = jumps.shape
    return [[synth.limbs_to_int(jumps[k, d]) for d in range(dp1)] for k in range(n)]


def _check(out, dist, jumps, threads, steps, bits):
    table = _table(dist, jumps)
    for g in threads:
        want = knots.accumulate_wrapped(dist, table, int(g), steps, bits)
        got = [synth.limbs_to_int(out[g, d]) for d in range(len(want))]
        assert got == want, (bits, int(g))


@pytest.mark.parametrize("bits", [32, 64, 96, 128])
@pytest.mark.parametrize("D", [1, 2, 3, 4, 5, 6])
def test_every_accumulator_matches_oracle(bits, D):
    # 300 accumulators: one full work-group of 256 and a ragged second one
    dist, jumps = synth.bit_tables(seed=20 + D, n_table=37, degree=D, bits=bits)
    out, ms = L.sph_hoa_accumulate_bits(bits, D, dist, jumps, 300, 32)
    assert ms >= 0.0
    _check(out, dist, jumps, range(300), 32, bits)


@pytest.mark.parametrize("bits", [32, 64, 128])
def test_benchmark_launch_sampled(bits):
    """The launch the benchmark times (2^20 accumulators, 1024 knots each, D = 3), on a sample of
    accumulators spread over the grid, the first and the last included."""
    dist, jumps = synth.bit_tables(seed=6, n_table=37, degree=3, bits=bits)
    n = 1 << 20
    out, _ = L.sph_hoa_accumulate_bits(bits, 3, dist, jumps, n, 1024)
    rng = np.random.default_rng(bits)
    sample = np.concatenate([[0, 255, 256, n - 1], rng.integers(0, n, 12)])
    _check(out, dist, jumps, sample, 1024, bits)


def test_single_entry_table_and_minimum_steps():
    dist, jumps = synth.bit_tables(seed=3, n_table=1, degree=2, bits=96)
    out, _ = L.sph_hoa_accumulate_bits(96, 2, dist, jumps, 5, 4)
    _check(out, dist, jumps, range(5), 4, 96)


def test_argument_errors():
    dist, jumps = synth.bit_tables(seed=3, n_table=4, degree=2, bits=64)
    with pytest.raises(L.SphHoaError):
        L.sph_hoa_accumulate_bits(48, 2, dist, jumps[:, :, :1], 8, 8)
    with pytest.raises(L.SphHoaError):
        L.sph_hoa_accumulate_bits(64, 2, dist, jumps, 8, 6)   # steps not a multiple of 4
    with pytest.raises(L.SphHoaError):
        L.sph_hoa_accumulate_bits(64, 2, dist, jumps, 0, 8)   # no accumulators
    d7, j7 = synth.bit_tables(seed=3, n_table=4, degree=7, bits=64)
    with pytest.raises(L.SphHoaError):
        L.sph_hoa_accumulate_bits(64, 7, d7, j7, 8, 8)
