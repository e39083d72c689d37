"""Peak-rate probes (measurement helpers): lane-operation counts, plausible
rates against the published MI355X figures, argument errors."""
import pytest

from paper_2111_13628_amd import nmc

pytestmark = pytest.mark.gpu

# 256 CUs x 64 lanes per clock x 2.4 GHz
VALU_PEAK = 256 * 64 * 2.4e9


def say(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("which", ["lds_distinct", "lds_random", "valu_int"])
def test_probe_counts_and_rates(which):
    say(f"case: probe {which}")
    iters, blocks = 512, 512
    ms, ops = nmc.probe_peak(which, iters, blocks)
    assert ops == blocks * 1024 * iters * (8 if which == "valu_int" else 16)
    assert ms > 0
    rate = ops / (ms / 1e3)
    # plausibility only: the rates are reported, not held to a figure
    assert 1e11 < rate < 4 * VALU_PEAK


def test_probe_argument_errors():
    say("case: probe argument errors")
    for which, iters, blocks in ((3, 8, 1), (-1, 8, 1), (0, 12, 1), (0, 0, 1), (2, 8, 0), (2, 1 << 25, 1)):
        with pytest.raises(nmc.NmcError) as e:
            nmc.probe_peak(which, iters, blocks)
        assert e.value.code == -1
