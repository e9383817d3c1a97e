"""Host logic of bench.py (no GPU): the one-GPU refusal, the measured-traffic records
(used only while the kernel source they were measured on is unchanged) and the
algorithmic bytes of each stage."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "..")


def _bench():
    spec = importlib.util.spec_from_file_location("bench_host_under_test",
                                                  os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 2
    assert "one GPU" in out.stderr


def test_traffic_records_follow_their_sources(monkeypatch):
    b = _bench()
    for kernel, rec in b.MEASURED_TRAFFIC.items():
        src, _, fkib, wkib, fs, ws = rec
        assert os.path.exists(os.path.join(ROOT, src)), src
        got = b.traffic_bytes(kernel)
        if got is not None:  # recorded on the current source: bytes = scaled counters
            assert got == (fkib * fs + wkib * ws) * 1024.0
    src, digest, fkib, wkib, fs, ws = b.MEASURED_TRAFFIC["smooth"]
    monkeypatch.setitem(b.MEASURED_TRAFFIC, "smooth", (src, "0" * 64, fkib, wkib, fs, ws))
    assert b.traffic_bytes("smooth") is None  # a changed kernel has no measured traffic
    assert b.traffic_bytes("no such kernel") is None


def test_stage_bytes():
    b = _bench()
    npart, ncell, cycles = 1000, 512, 6
    plain = b.stage_bytes(npart, ncell, cycles)
    chained = b.stage_bytes(npart, ncell, cycles, chained=True)
    assert plain["ms_drift"] == 68.0 * npart and chained["ms_drift"] == 0.0
    assert plain["ms_deposit"] == chained["ms_deposit"] == 16.0 * npart + 4.0 * ncell
    # 82 B/cell per V-cycle (2 + 2 sweeps, transfers, all levels, finest norm) and the
    # two sweeps of the last norm pass, whose output is kept
    assert plain["ms_solve"] == chained["ms_solve"] == (cycles * 82.0 + 24.0) * ncell
    assert plain["ms_interp"] == 52.0 * npart + 4.0 * ncell
    assert chained["ms_interp"] == 60.0 * npart + 4.0 * ncell
