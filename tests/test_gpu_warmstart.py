"""What the trained warm-start network gains over the method without it.

Uses the committed network (trained on the GPU by the library's own
kernels on converged amplitudes of 512 synthetic systems, seeds 50000..50511,
with `python -m paper_2004_03682_amd.warmstart train`) on held-out systems of
the same distribution (seeds 40000..), and checks that the MP2 start stays
the fallback: a network that predicts nonsense is rejected system by system
and the iteration then matches the plain MP2 start."""
import numpy as np
import pytest

import fsgen

pytestmark = pytest.mark.gpu


def _held_out(n=8):
    ss = fsgen.batch_systems(64, 40000)
    ss = sorted(ss, key=lambda s: s.nocc ** 2 * s.nvirt ** 4 / s.nirrep)[:n]     # the cheapest ones
    return ss


def test_trained_network_saves_iterations():
    import paper_2004_03682_amd as F
    from paper_2004_03682_amd import warmstart as W
    b = W.make_batch(_held_out())
    net = F.MLP(0)
    meta = W.load(net)
    print("network:", {k: float(v) for k, v in meta.items()}, flush=True)
    out = W.evaluate(net, b, log=print)
    assert out["both_converged"] == b.nsys
    assert out["max_abs_dE_mp2_vs_learned"] <= 2e-9
    assert out["fallback_systems"] == 0
    # fewer iterations to |E - E_final| < 1e-8 Eh on average, start-up evaluations included
    assert out["iterations_to_1e-8_learned_mean"] < out["iterations_to_1e-8_mp2_mean"]
    # The time to 1e-8 Eh is reported, not asserted: on these eight smallest
    # systems the network's start evaluations cost about what the saved
    # fraction of an iteration saves (measured 0.027 s MP2 start, 0.028 s
    # learned); on the 64-system batch of the benchmark the learned start
    # reaches 1e-8 Eh 2 % sooner on average.
    print("seconds to 1e-8 Eh (mean): MP2", out["seconds_to_1e-8_mp2_mean"], "learned",
          out["seconds_to_1e-8_learned_mean"], flush=True)
    b.destroy()


def test_bad_network_falls_back_to_the_mp2_start():
    import paper_2004_03682_amd as F
    from paper_2004_03682_amd import warmstart as W
    b = W.make_batch(_held_out(4))
    net = F.MLP(0)
    p = np.random.default_rng(0).normal(size=net.n_params).astype(np.float32) * 3.0
    net.set_params(p)
    out = W.evaluate(net, b, log=print)
    assert out["fallback_systems"] == b.nsys
    assert out["both_converged"] == b.nsys
    assert out["max_abs_dE_mp2_vs_learned"] <= 2e-9
    # after the rejected first iteration the systems iterate like the MP2 start
    assert out["iterations_learned_mean"] <= out["iterations_mp2_mean"] + 4
    b.destroy()
