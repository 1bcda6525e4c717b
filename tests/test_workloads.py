"""The physics switches of the paper's comparisons (Sec. V) on the oracle (CPU)."""
import numpy as np

import workloads as W


def test_variant_switches(oracle_lib):
    base = W.config0(n_primaries=1500, n_steps=60)
    t0 = base.instances[0].T.copy()
    names = oracle_lib.COUNTER_NAMES
    # transparent interfaces: every interface hit transmits
    tr = W.variant(base, transparent=True)
    c = oracle_lib.run(tr).counters
    assert c[:, names.index("refl_if")].sum() == 0 and c[:, names.index("transmit")].sum() > 0
    # an elastic channel of 30 fs in every layer
    el = W.variant(base, tau_el=30.0)
    c = oracle_lib.run(el).counters
    assert c[:, names.index("ev_el")].sum() > 0
    # no secondaries
    ns = W.variant(base, secondaries=False)
    c = oracle_lib.run(ns).counters
    assert c[:, names.index("spawned")].sum() == 0
    # the original is untouched
    assert np.array_equal(base.instances[0].T, t0)
    assert base.secondaries and not base.absorb_next and not base.gen_moment
    assert np.all(base.instances[0].inv_tau_el == 0)
