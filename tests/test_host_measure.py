"""Host-side checks of the measurement tooling (no GPU): the bench's one-GPU
contract, kernel-name shortening in the profile summaries, and the rule that
HBM traffic is read only from a counter summary taken on the current kernel
source."""
import os
import subprocess
import sys

from paper_2410_15519_amd import profsum

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_short_kernel_names():
    assert profsum.short_name("void ctd::k_cubic_g<float>(ctd::DevInst, int)") == "k_cubic_g<float>"
    assert profsum.short_name("ctd::(anonymous namespace)::k_gemm64(ctd::GemmArgs)") == "k_gemm64"
    assert profsum.short_name("k_copy16") == "k_copy16"


def _summary(tmp_path, sha, lines):
    p = tmp_path / "traffic.md"
    p.write_text("# t\n\nkernel source sha256 (first 16 hex): " + sha + "\n\n" + "\n".join(lines) + "\n")
    return str(p)


def test_traffic_read_only_for_current_kernel_source(tmp_path):
    cur = profsum.kernel_source_sha()
    lines = ["traffic_bytes_per_launch k_cubic_g<float> [245760] = 18508470",
             "traffic_bytes_per_launch k_fd_apply [65536] = 10738167"]
    p = _summary(tmp_path, cur, lines)
    assert profsum.traffic_from_summary(p, "k_cubic_g<float> [245760]") == 18508470.0
    assert profsum.traffic_from_summary(p, "k_fd_apply [65536]") == 10738167.0
    # another grid of the same kernel is another entry
    assert profsum.traffic_from_summary(p, "k_cubic_g<float> [20480]") is None
    # a summary taken on a different kernel source is not used
    stale = _summary(tmp_path, "0" * 16 if cur != "0" * 16 else "1" * 16, lines)
    assert profsum.traffic_from_summary(stale, "k_cubic_g<float> [245760]") is None
    assert profsum.traffic_from_summary(str(tmp_path / "missing.md"), "k_cubic_g<float> [245760]") is None


def test_committed_profiles_name_their_commands():
    """Every committed summary gives the command that made it and runs only
    committed files."""
    d = os.path.join(ROOT, "profiles")
    names = [n for n in os.listdir(d) if n.endswith(".md")]
    assert names
    for n in names:
        text = open(os.path.join(d, n)).read()
        assert "rocprofv3" in text, n
        assert "_work" not in text, n
