"""The allocation-free set-up (pic_init_static) against the workspace set-up (pic_init).

Both run the same problem through the C ABI; the binary64 bins (exact conversions of the
integer bins) and the per-step counters must be identical.  Two problems in a row on the
static workspace, the second smaller, so that the second run starts from the first one's
leftovers in the array."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    return torch


def _run(problem, static, tuning=None):
    from paper_1807_04733_amd import PicSim
    sim = PicSim(problem, device="cuda:0", static_workspace=static, tuning=tuning)
    try:
        sim.step()
        cnt = sim.counters()
        dens, cur = sim.deposit()
        return cnt, [d.cpu().numpy() for d in dens], [c.cpu().numpy() for c in cur]
    finally:
        sim.close()


def _same(a, b):
    ca, da, ua = a
    cb, db, ub = b
    assert np.array_equal(ca, cb)
    for x, y in zip(da, db):
        assert np.array_equal(x, y)
    for x, y in zip(ua, ub):
        assert np.array_equal(x, y)


def test_static_workspace_matches_workspace_setup(torch_gpu):
    from paper_1807_04733_amd.sim import workspace_bytes
    from paper_1807_04733_amd import _abi
    big = W.config1(parallel=False, n_primaries=20000, n_steps=160)
    small = W.config0(n_primaries=3000, n_steps=70)
    assert workspace_bytes(small) < workspace_bytes(big) <= _abi.STATIC_WORKSPACE_BYTES
    for prob in (big, small):
        print(f"static workspace vs pic_init: {prob.name}", flush=True)
        ref = _run(prob, static=False)
        got = _run(prob, static=True)
        _same(got, ref)
        assert ref[0][:, 9].sum() > 0
    # two-step launches on the static workspace as well
    ref = _run(small, static=False, tuning=dict(sub_steps=2, z_every=4))
    got = _run(small, static=True, tuning=dict(sub_steps=2, z_every=4))
    _same(got, ref)


def test_static_workspace_limits(torch_gpu):
    from paper_1807_04733_amd import PicSim, PicError, _abi
    from paper_1807_04733_amd.sim import workspace_bytes
    huge = W.config1(n_primaries=2_000_000, n_steps=200)
    assert workspace_bytes(huge) > _abi.STATIC_WORKSPACE_BYTES
    with pytest.raises(PicError) as e:
        PicSim(huge, device="cuda:0", static_workspace=True)
    assert e.value.code == 2                       # PIC_ENOMEM
    small = W.config0(n_primaries=500, n_steps=10)
    first = PicSim(small, device="cuda:0", static_workspace=True)
    try:
        with pytest.raises(PicError) as e:
            PicSim(small, device="cuda:0", static_workspace=True)
        assert e.value.code == 5                   # PIC_ESTATE: the array is taken
    finally:
        first.close()
    again = PicSim(small, device="cuda:0", static_workspace=True)
    again.close()
