"""bench.py's command-line contract on a host without a GPU (more than one
GPU is refused with a message and a non-zero status, before anything touches
a device), and the reading of the profile summaries it cites."""
import os
import subprocess
import sys

import pytest

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


def test_profile_launch_sequences():
    # label=regex@start:count picks count consecutive matches from start
    # (negative: from the end), and refuses a range the run does not hold
    from paper_2403_18661_amd import profsum
    (label, rx, start, count), = profsum._seqs(["bf16_layers=conv<P,@-4:2"])
    assert (label, start, count) == ("bf16_layers", -4, 2)
    rows = [{"Kernel_Name": n} for n in ("conv<P,a>", "stem", "conv<P,b>", "conv<P,c>", "conv<P,d>", "conv<Q,e>")]
    assert [r["Kernel_Name"] for r in profsum._slice(rows, rx, start, count)] == ["conv<P,a>", "conv<P,b>"]
    assert [r["Kernel_Name"] for r in profsum._slice(rows, rx, -2, 2)] == ["conv<P,c>", "conv<P,d>"]
    with pytest.raises(ValueError):
        profsum._slice(rows, rx, -5, 2)
    with pytest.raises(ValueError):
        profsum._seqs(["x=y@0:0"])
    assert profsum._short("void afm::conv_mfma_kernel<afm::PBF16, 7, 1>(afm::ConvArgs)") == "PBF16,7,1"
