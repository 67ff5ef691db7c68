"""bench.py's command-line contract on a host without a GPU: more than one
GPU is refused with a message and a non-zero status, before anything touches
a device."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=600, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
    assert r.stdout.strip() == "" or not r.stdout.strip().startswith("{")   # no result line


def test_profile_traffic_is_dropped_when_its_sources_change(tmp_path):
    # a summary's figures count only while the kernel sources it names are
    # unchanged; sources it does not name may change freely
    sys.path.insert(0, ROOT)
    from paper_2403_18661_amd import profsum
    srcs = ("csrc/whiten.hip", "csrc/psd.hip")
    body = ("groups (last N dispatches):\n  label N avg_ms fetch_MB write_MB traffic\n"
            "  whiten 3 1.3 3185.0 1414.0 4600000000\n\n")
    good = tmp_path / "good.txt"
    good.write_text(body + "source_files " + " ".join(srcs) + "\nsource_sha256 " + profsum.source_sha256(srcs) + "\n")
    assert profsum.read_traffic(str(good))["whiten"]["traffic"] == 4.6e9
    stale = tmp_path / "stale.txt"
    stale.write_text(body + "source_files " + " ".join(srcs) + "\nsource_sha256 " + "0" * 64 + "\n")
    assert profsum.read_traffic(str(stale)) == {}
    foreign = tmp_path / "foreign.txt"   # a file that is not a kernel source is never trusted
    foreign.write_text(body + "source_files bench.py\nsource_sha256 " + profsum.source_sha256(srcs) + "\n")
    assert profsum.read_traffic(str(foreign)) == {}
