"""The vector-ALU issue-rate probe (a measurement helper of the roofline)."""
import pytest

pytestmark = pytest.mark.gpu


def test_valu_probe_rates_are_plausible():
    from paper_2605_18566_amd import probe_valu_rate
    r1, g1 = probe_valu_rate(1, iters=4000)
    r8, g8 = probe_valu_rate(8, iters=4000)
    print(f"1 wave/SIMD: {r1:.3f} per CU-clock at {g1:.3f} GHz; 8 waves/SIMD: {r8:.3f} at {g8:.3f} GHz", flush=True)
    # the shader clock of an MI355X is at most 2.4 GHz; the FP32 peak is 2.0 wave-level FMAs per CU-clock
    for g in (g1, g8):
        assert 0.5 < g < 3.0
    for r in (r1, r8):
        assert 0.05 < r < 2.2
    assert r8 >= r1


def test_valu_probe_rejects_bad_arguments():
    from paper_2605_18566_amd import _lib, probe_valu_rate
    with pytest.raises(_lib.HJGError):
        probe_valu_rate(0)
    with pytest.raises(_lib.HJGError):
        probe_valu_rate(9)
    with pytest.raises(_lib.HJGError):
        probe_valu_rate(1, form=13)
