"""The tuning table compiled into the library: well-formed and covering every case."""
import os
import re

from conftest import ROOT

INC = os.path.join(ROOT, "paper_2105_07298_amd", "csrc", "tune_table.inc")


def entries():
    text = open(INC).read()
    apsp = re.search(r"kTuneApsp\[\] = \{(.*?)\};", text, re.S).group(1)
    batched = re.search(r"kTuneBatched\[\] = \{(.*?)\};", text, re.S).group(1)
    rows = []
    for m in re.finditer(r"\{([^{}]*)\}", apsp):
        f = [x.strip() for x in m.group(1).split(",")]
        hi = (1 << 40) if "<<" in f[3] else int(f[3])
        rows.append((int(f[0]), int(f[1]), int(f[2]), hi, int(f[4]), int(f[5]), int(f[6]), int(f[7]), int(f[8])))
    brows = [tuple(int(x.strip().rstrip("ul"), 0) for x in m.group(1).split(","))
             for m in re.finditer(r"\{([^{}]*)\}", batched)]
    return rows, brows


def test_apsp_table_covers_every_size_once():
    import paper_2105_07298_amd as fw
    rows, _ = entries()
    dtypes = (fw.FW_F32, fw.FW_F64, fw.FW_F16)
    supported = {dt: set(fw.fw_list_configs(dt)) for dt in dtypes}
    assert {r[0] for r in rows} == set(dtypes)
    for dt in dtypes:
        for path in (0, 1):
            rs = sorted((r for r in rows if r[0] == dt and r[1] == path), key=lambda r: r[2])
            assert rs, (dt, path)
            assert rs[0][2] == 0 and rs[-1][3] >= (1 << 40)
            for a, b in zip(rs[:-1], rs[1:]):
                assert a[3] == b[2], "size ranges must tile [0, inf)"
            for r in rs:
                assert (r[4], r[5], r[6], r[7]) in supported[dt], r
                assert r[8] in (fw.FW_SCHED_SERIAL, fw.FW_SCHED_LOOKAHEAD, fw.FW_SCHED_PAIRS,
                                fw.FW_SCHED_PAIRS_LOOKAHEAD), r


def test_batched_table_complete():
    _, brows = entries()
    keys = {(b[0], b[1]) for b in brows}
    assert keys == {(0, 0), (0, 1), (1, 0), (1, 1)}
    # tile64 masks: 64 x 64 tiles never for n <= 32 (they would pad it to 64),
    # always above the 768 vertices the tuner times
    assert all(0 <= b[2] < (1 << 64) and not (b[2] & 1) for b in brows)
    assert all((b[2] >> 24) == (1 << 40) - 1 for b in brows)
