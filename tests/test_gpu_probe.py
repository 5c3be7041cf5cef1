"""Matrix-core throughput probe (fscc_probe_mfma): each kind reports a rate
between 30 % and 110 % of the MI355X spec-sheet dense peak of its
instruction and a longer run takes proportionally longer (its argument
checks run on the host: test_abi.py)."""
import pytest

pytestmark = pytest.mark.gpu

SPEC = {"fp64": 78.6, "bf16": 2500.0, "fp32": 157.3}   # TFLOP/s


@pytest.mark.parametrize("kind", ["fp64", "bf16", "fp32"])
def test_probe_rate_is_a_plausible_fraction_of_the_spec_peak(kind):
    import paper_2004_03682_amd as F
    tf, ms = F.probe_mfma(kind, 4096)
    print(kind, f"{tf:.1f} TFLOP/s ({tf / SPEC[kind]:.3f} of spec) in {ms:.3f} ms", flush=True)
    assert 0.3 * SPEC[kind] <= tf <= 1.1 * SPEC[kind]
    tf2, ms2 = F.probe_mfma(kind, 8192)
    assert 1.6 <= ms2 / ms <= 2.4        # the time is the MFMA chains', not launch overhead
    assert abs(tf2 / tf - 1.0) <= 0.25
