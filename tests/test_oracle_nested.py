"""The nested CPU comparator (events in flight x FED ranges) gives the oracle's own results."""
import numpy as np
import pytest

import fedgen
import oracle
from oracle.nested import NestedRunner, fed_ranges, process_event_ranges


@pytest.mark.parametrize("m", [1, 3, 7, 50])
@pytest.mark.parametrize("cfg_id", [0, 4])
def test_fed_ranges_give_the_whole_event(cfg_id, m):
    cfg = fedgen.CONFIGS[cfg_id].with_(n_fed=50)
    cal = fedgen.make_calibration(cfg)
    ev = fedgen.make_event(cfg, cal, 2)
    whole = oracle.process_event(ev.zs, ev.fed_offset, cal.noise, cal.gain, cal.bad)
    parts = process_event_ranges(ev.zs, ev.fed_offset, cal.noise, cal.gain, cal.bad, m)
    assert parts.cl.tobytes() == whole.cl.tobytes()
    assert parts.adc.tobytes() == whole.adc.tobytes()


def test_ranges_cover_every_fed_once():
    for n, m in ((440, 16), (50, 7), (5, 9), (1, 4)):
        r = fed_ranges(n, m)
        assert r[0][0] == 0 and r[-1][1] == n
        assert all(a < b for a, b in r) and all(r[i][1] == r[i + 1][0] for i in range(len(r) - 1))


def test_runner_counts_events():
    cfg = fedgen.CONFIGS[0].with_(n_fed=20)
    cal = fedgen.make_calibration(cfg)
    evs = fedgen.make_events(cfg, cal, range(3))
    done, secs, lat = NestedRunner(evs, cal, 2, 3).run(0.3)
    assert done >= 2 and len(lat) == done and secs > 0
