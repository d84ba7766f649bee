"""The device-error path of the ordered look-back, forced from the host.

A look-back wait is bounded; a wait that reaches its bound reports a stall
through the host-mapped error word and raises the launch's abort flag, so
that every other wait of the launch ends at once, and the next call on the
device returns PRNGD_ERR_DEVICE.  A correct launch never stalls, so the
test lowers the bound (prngd_probe_set_spin_limit) to a poll or two, which
makes waits that would finish end early instead: every kernel still exits
normally.  Then the bound is restored and the library fills correctly again.
"""
import numpy as np
import pytest

import oracle as O
from gpu_util import note

torch = pytest.importorskip("torch")
from paper_1401_8230_amd import prngd  # noqa: E402

pytestmark = pytest.mark.gpu


def test_a_stalled_look_back_surfaces_as_a_device_error():
    prngd.set_tuning("philox", 8, path="ordered")
    g = prngd.Generator(5, "philox", w=8)
    out = torch.empty(1 << 24, dtype=torch.float64, device="cuda:0")
    seen = None
    try:
        prngd.probe_set_spin_limit(1)
        for attempt in range(3):
            note(f"look-back with a one-poll bound, attempt {attempt}")
            try:
                g.fill(out)
                torch.cuda.synchronize()
            except prngd.PrngdError as e:       # reported by this call: a previous stall
                seen = e
                break
    finally:
        prngd.probe_set_spin_limit(0)
    if seen is None:
        note("the default bound again; the next call reports the stall")
        try:
            g.fill(out[:10])
            torch.cuda.synchronize()
        except prngd.PrngdError as e:
            seen = e
    assert seen is not None, "no stall was reported"
    assert seen.status == prngd.ERR_DEVICE
    # reported once: the library goes on, and fills are exact again
    note("after the reported stall")
    g.set_position(3, 1000)
    g.fill(out[:100003])
    torch.cuda.synchronize()
    ref = O.PRNGD(O.GEN_PHILOX, 8, seed=5, stream=3, counter=1000)
    assert np.array_equal(out[:100003].cpu().numpy().view(np.uint64), ref.fill(100003).view(np.uint64))
    assert g.get_position() == (3, ref.counter)
    g.close()
    prngd.reset_tuning("philox", 8)
