"""The serving loop's scheduler (admission by device-memory budget, slots,
release of idle arenas, wake-ups, bounded waits) on the host, with a mock
device side: tests/server_replay.cpp drives the library's own scheduler and
workspace bound with the serving workload's request stream (Poisson arrivals
at 20/s, mixed QEP / delay / BEM requests), each request sleeping for a
modelled latency.  Built with g++ (once plain, once with ThreadSanitizer);
no GPU is involved."""
import os
import shutil
import subprocess

import pytest

import nep_inputs as ni

HERE = os.path.dirname(os.path.abspath(__file__))
FAMILY = {"qep": 0, "delay": 1, "bem": 2}


def _build(tmp_path, sanitize):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / ("replay_tsan" if sanitize else "replay"))
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-pthread", os.path.join(HERE, "server_replay.cpp"), "-o", exe]
    if sanitize:
        cmd.insert(1, "-fsanitize=thread")
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return exe


def _stream(count):
    reqs = ni.config_c4(count=count)
    return "".join(f"{r['t']:.6f} {FAMILY[r['family']]} {r['n']} {r['N']} {r['L']}\n" for r in reqs)


def _replay(exe, count, budget_gib, slots, scale, timeout=300):
    inp = f"{budget_gib} {slots} {scale} 0\n" + _stream(count)
    p = subprocess.run([exe], input=inp, capture_output=True, text=True, timeout=timeout)
    summary = [l for l in p.stdout.splitlines() if l.startswith("summary")]
    print(p.stdout[-3000:], p.stderr[-3000:])
    return p.returncode, (summary[0] if summary else ""), p.stderr


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    return _build(tmp_path_factory.mktemp("replay"), sanitize=False)


def test_replay_first_48_requests(exe):
    # the 48 requests whose replay on the device stopped after 30 results
    rc, summary, _ = _replay(exe, 48, 200.0, 4, 0.05)
    assert rc == 0, summary
    assert "48 done" in summary and "over budget 0" in summary


def test_replay_full_stream(exe):
    # all 600 requests of the serving workload, time compressed
    rc, summary, _ = _replay(exe, 600, 200.0, 4, 0.004)
    assert rc == 0, summary
    assert "600 done" in summary


def test_replay_tight_budget_many_slots(exe):
    # a budget a few requests fill: slots must give idle arenas back and wake
    # each other, and the held memory must stay within the budget
    rc, summary, _ = _replay(exe, 120, 48.0, 8, 0.01)
    assert rc == 0, summary
    assert "over budget 0" in summary


def test_replay_under_thread_sanitizer(tmp_path):
    exe = _build(tmp_path, sanitize=True)
    rc, summary, err = _replay(exe, 64, 64.0, 6, 0.01)
    assert "ThreadSanitizer" not in err, err[-4000:]
    assert rc == 0, summary
