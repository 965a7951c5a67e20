"""Call tracing (SHT_TRACE): one stderr line per traced entry point with its arguments, status
and host time.  The calls here fail their argument checks before touching a device, so the
test runs without a GPU."""
import ctypes

from paper_0910_5435_amd import _lib


def test_trace_lines_follow_the_environment(capfd, monkeypatch):
    lib = _lib.load()
    out = ctypes.c_void_p()
    monkeypatch.delenv("SHT_TRACE", raising=False)
    assert lib.sht_plan_ex(3, 1e-12, None, ctypes.byref(out)) == _lib.SHT_EUNSUPPORTED
    assert capfd.readouterr().err == ""
    monkeypatch.setenv("SHT_TRACE", "1")
    assert lib.sht_plan_ex(3, 1e-12, None, ctypes.byref(out)) == _lib.SHT_EUNSUPPORTED
    assert lib.sht_synth(None, None, None, 1, None, 0, None) == _lib.SHT_EINVAL
    assert lib.sht_order_plan(8, 2.0, None, ctypes.byref(out)) == _lib.SHT_EINVAL
    assert lib.sht_batch_create(None, 0, 0, 0, 0, None, ctypes.byref(out)) == _lib.SHT_EINVAL
    err = capfd.readouterr().err.splitlines()
    assert len(err) == 4, err
    assert err[0].startswith("sht: sht_plan_ex(l=3, eps=1e-12, leaf_width=0, precision=0, id_device=0) -> -4 (")
    assert err[1].startswith("sht: sht_synth(l=0, F=1, precision=0) -> -1 (")
    assert err[2].startswith("sht: sht_order_plan(l=8, eps=2, leaf_width=0) -> -1 (")
    assert err[3].startswith("sht: sht_batch_create(nreq=0, op=0, precision=0) -> -1 (")
    assert all(", host " in e and e.endswith(" ms") for e in err)
    monkeypatch.setenv("SHT_TRACE", "0")
    assert lib.sht_plan_ex(3, 1e-12, None, ctypes.byref(out)) == _lib.SHT_EUNSUPPORTED
    assert capfd.readouterr().err == ""
