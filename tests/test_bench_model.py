"""Host logic of the benchmark's byte models (no GPU): the method's bytes per particle-step
and the two-step kernel's own bytes, on hand-made counters."""
import numpy as np

import bench


def _counters(rows):
    c = np.zeros((len(rows), 12), np.int64)
    for n, r in enumerate(rows):
        for k, v in r.items():
            c[n, k] = v
    return c


def test_method_bytes_by_hand():
    # step 0: 10 primaries injected, 10 alive after; step 1: 2 events (1 inelastic with a
    # secondary, 1 elastic), 3 reflections and 4 transmissions, 11 alive after
    cnt = _counters([{0: 10, 9: 10}, {1: 1, 2: 1, 3: 1, 7: 2, 8: 1, 6: 4, 9: 11}])
    one = np.array([[0, 0, 0, 0, 0, 1], [0, 0, 0, 0, 1, 1]], float)
    b = bench.method_bytes(cnt, False, one)
    # FP32: state 24 B + z 4 B per particle-step, 8 B per event, 4 B per reflection and
    # 24 B per created carrier; transmissions move nothing
    assert b[0] == 10 * 28 + 10 * 24
    assert b[1] == 10 * 28 + 2 * 8 + 3 * 4 + 1 * 24
    both = bench.method_bytes(cnt, False, np.array([[0, 0, 0, 0, 0, 2]], float))
    assert both[0] == b.sum()
    b64 = bench.method_bytes(cnt, True, one)
    assert b64[1] == 10 * 40 + 2 * 12 + 3 * 8 + 1 * 32


def test_two_step_kernel_moves_less_than_the_method():
    # 100 carriers for 8 steps, nothing happening: the method moves 28 B per particle-step;
    # two steps per launch with z written every 8 steps read 24 B once per launch and write
    # z once
    cnt = _counters([{0: 100, 9: 100}] + [{9: 100}] * 7)
    rows = np.array([[0, 0, 0, 0, 2 * k, 2] for k in range(4)], float)
    m = bench.method_bytes(cnt, False, rows).sum()
    k = bench.alg_bytes(cnt, False, launches=rows, z_every=8, sub_steps=2).sum()
    assert m == 8 * 100 * 28 + 100 * 24
    assert k == 3 * 100 * 24 + 100 * 4 + 100 * 24
    assert k < m
