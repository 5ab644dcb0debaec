"""The C-ABI library: loads, exports every declared symbol, rejects bad arguments
before touching a device.  CPU-only (no kernel is launched)."""
import ctypes
import os
import re

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "fw_apsp.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fw_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def fw():
    import paper_2105_07298_amd as fw
    fw.lib()
    return fw


def test_every_declared_symbol_is_exported(fw):
    names = declared_functions()
    assert "fw_apsp" in names and "fw_apsp_batched" in names and "fw_apsp_backward" in names
    L = ctypes.CDLL(fw._lib.LIB_PATH)
    for name in names:
        assert hasattr(L, name), f"{name} declared in fw_apsp.h but not exported"
    assert set(names) == set(fw._lib.EXPORTS)


def test_status_strings(fw):
    assert fw.fw_status_string(0) == "ok"
    for st in (-1, -2, -3, -4, -5):
        assert fw.fw_status_string(st) not in ("ok", "unknown status")
    assert fw.fw_status_string(17) == "unknown status"
    assert "gfx950" in fw.fw_version()


def call_raw(fw, *args):
    return fw.lib().fw_apsp(*args)


@pytest.mark.parametrize("args", [
    (0, 0, 4096, None, None),          # n = 0
    (0, -5, 4096, None, None),         # n < 0
    (0, (1 << 20) + 1, 4096, None, None),  # n too large
    (0, 16, None, None, None),         # null dist
    (7, 16, 4096, None, None),         # unknown dtype
])
def test_invalid_arguments(fw, args):
    st = call_raw(fw, *args)
    assert st == fw.FW_EINVAL
    assert fw.fw_last_error() != ""


def test_invalid_config(fw):
    L = fw.lib()
    for bad in ((64, 96, 64, 1),     # tile edge not compiled
                (64, 32, 256, 1),    # a wave-row tile asked of the LDS-panel kernel
                (64, 128, 128, 2),   # an LDS-panel tile asked of the wave-row kernel
                (32, 64, 128, 2)):   # wave-row tile rows must divide the block
        cfg = fw._lib.FwConfig(*bad)
        assert L.fw_apsp_config(0, 128, 4096, None, ctypes.byref(cfg), None) == fw.FW_EUNSUPPORTED, bad
        assert "not compiled in" in fw.fw_last_error()
    for bad in ((64, 64, 64, 3), (-1, 64, 64, 1), (64, 64, -64, 0), (64, 64, 64, 1, 5), (64, 64, 64, 1, -1)):
        cfg = fw._lib.FwConfig(*bad)
        assert L.fw_apsp_config(0, 128, 4096, None, ctypes.byref(cfg), None) == fw.FW_EINVAL, bad


def test_list_configs(fw):
    for dt in (0, 1):
        cfgs = fw.fw_list_configs(dt)
        assert len(cfgs) == len(set(cfgs)) >= 10
        assert {c[3] for c in cfgs} == {fw.FW_P4_PANELS, fw.FW_P4_WAVEROWS}
        for b, tm, tn, var in cfgs:
            assert b in (32, 64)
            if var == fw.FW_P4_PANELS:
                assert tm in (64, 128) and tn in (64, 128) and tm % b == 0 and tn % b == 0
            else:
                assert b % tm == 0 and tm % 4 == 0 and tn in (64, 128, 256)
                if dt == 1:
                    assert tn <= 128  # 16-byte lane vectors hold 2 doubles
    assert fw.lib().fw_list_configs(7, None, 0) == fw.FW_EINVAL
    assert fw.lib().fw_list_configs(0, None, 3) == fw.FW_EINVAL


def test_list_configs_f16(fw):
    """binary16: LDS-panel kernels only, 8 columns per thread (tile_n >= 128)."""
    cfgs = fw.fw_list_configs(fw.FW_F16)
    assert len(cfgs) == len(set(cfgs)) >= 4
    for b, tm, tn, var in cfgs:
        assert var == fw.FW_P4_PANELS and b in (32, 64)
        assert tn in (128, 256) and tm % 16 == 0 and tn % b == 0
    L = fw.lib()
    for bad in ((64, 64, 64, 1), (64, 64, 128, 2)):
        cfg = fw._lib.FwConfig(*bad)
        assert L.fw_apsp_config(fw.FW_F16, 128, 4096, None, ctypes.byref(cfg), None) == fw.FW_EUNSUPPORTED, bad


def test_f16_only_where_declared(fw):
    """FW_F16 is an fw_apsp dtype; the batched, backward and out-of-core entry
    points refuse it before touching a device."""
    import numpy as np
    L = fw.lib()
    ns = np.array([4], dtype=np.int32)
    offs = np.array([0], dtype=np.int64)
    assert L.fw_apsp_batched(fw.FW_F16, 1, ns.ctypes.data, offs.ctypes.data, 4096, None, None) == fw.FW_EINVAL
    assert "FW_F16" in fw.fw_last_error()
    assert L.fw_apsp_backward(fw.FW_F16, 16, 1, 4096, 4096, 4096, 4096, None) == fw.FW_EINVAL
    assert L.fw_apsp_ooc(fw.FW_F16, 16, 4096, None, 1 << 20, None) == fw.FW_EINVAL
    assert L.fw_ooc_superblock(fw.FW_F16, 3000, 0, 1 << 30) == fw.FW_EINVAL
    assert L.fw_apsp(3, 16, 4096, None, None) == fw.FW_EINVAL


def test_query_config(fw):
    for dt in (0, 1, 2):
        compiled = set(fw.fw_list_configs(dt))
        for n in (1, 100, 1000, 5000, 16384, 65536):
            for path in (False, True):
                q = fw.fw_query_config(dt, n, path)
                assert q[:4] in compiled and q[4] in (fw.FW_SCHED_SERIAL, fw.FW_SCHED_LOOKAHEAD, fw.FW_SCHED_PAIRS,
                                                                    fw.FW_SCHED_PAIRS_LOOKAHEAD)


@pytest.mark.skipif(os.path.exists("/dev/kfd"), reason="a GPU is present: would launch on a bogus pointer")
def test_no_device_reports_hip_error(fw):
    st = call_raw(fw, 0, 16, 4096, None, None)
    assert st == fw.FW_EHIP
    assert fw.fw_last_error()


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    import paper_2105_07298_amd._lib as L
    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(ImportError):
        L.lib()


def test_batched_argument_errors_before_device(fw):
    import numpy as np
    L = fw.lib()
    ns = np.array([4, 0], dtype=np.int32)
    offs = np.array([0, 16], dtype=np.int64)
    assert L.fw_apsp_batched(0, 2, ns.ctypes.data, offs.ctypes.data, 4096, None, None) == fw.FW_EINVAL
    assert L.fw_apsp_batched(0, 0, ns.ctypes.data, offs.ctypes.data, 4096, None, None) == fw.FW_EINVAL
    assert L.fw_apsp_batched(0, 1, None, offs.ctypes.data, 4096, None, None) == fw.FW_EINVAL
    offs2 = np.array([-1], dtype=np.int64)
    ns2 = np.array([3], dtype=np.int32)
    assert L.fw_apsp_batched(0, 1, ns2.ctypes.data, offs2.ctypes.data, 4096, None, None) == fw.FW_EINVAL


def test_backward_argument_errors_before_device(fw):
    L = fw.lib()
    assert L.fw_apsp_backward(0, 5000, 1, 4096, 4096, 4096, 4096, None) == fw.FW_EINVAL
    assert L.fw_apsp_backward(0, 16, 1, 4096, None, 4096, 4096, None) == fw.FW_EINVAL
    assert L.fw_apsp_backward(0, 16, 0, 4096, 4096, 4096, 4096, None) == fw.FW_EINVAL
    assert L.fw_apsp_backward(3, 16, 1, 4096, 4096, 4096, 4096, None) == fw.FW_EINVAL


def test_ooc_superblock_choice(fw):
    """The super-block edge is the largest multiple of 256 whose working set fits
    the byte budget: 4 S^2 + 4 S ceil(n/S) S elements, and with the path matrix
    as many int32 labels plus S^2 more."""
    def need(n, S, es, path):
        nb = -(-n // S)
        blocks = 4 * S * S + 4 * S * nb * S
        return blocks * es + ((blocks + S * S) * 4 if path else 0)
    for dt, es in ((fw.FW_F32, 4), (fw.FW_F64, 8)):
        for path in (False, True):
            for n in (1, 300, 3000, 16384, 100000):
                for S_want in (256, 512, 1024, 4096):
                    budget = need(n, S_want, es, path)
                    S = fw.fw_ooc_superblock(dt, n, path, budget)
                    assert S % 256 == 0 and need(n, S, es, path) <= budget
                    top = -(-n // 256) * 256
                    assert S == top or need(n, S + 256, es, path) > budget
            assert fw.lib().fw_ooc_superblock(dt, 3000, 1 if path else 0, 1000) == fw.FW_ENOMEM
    assert fw.lib().fw_ooc_superblock(9, 3000, 0, 1 << 30) == fw.FW_EINVAL


def test_validate_argument_errors_before_device(fw):
    L = fw.lib()
    assert L.fw_validate_input(0, 0, 4096, None) == fw.FW_EINVAL
    assert L.fw_validate_input(0, 16, None, None) == fw.FW_EINVAL
    assert L.fw_validate_input(9, 16, 4096, None) == fw.FW_EINVAL
