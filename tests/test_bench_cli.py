"""The benchmark's command line on the CPU: more than one GPU is refused with
a message (the implementation runs on one GPU), and the help text lists the
contract's flags."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = run("--gpus", "2", "--steps", "1", "--warmup", "0")
    assert r.returncode == 2
    assert "single GPU" in r.stderr
    assert r.stdout == ""


def test_help_lists_contract_flags():
    r = run("--help")
    assert r.returncode == 0
    for flag in ("--gpus", "--steps", "--warmup"):
        assert flag in r.stdout


def _bench_module():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_traffic_lookup_by_tiling(tmp_path):
    """`roofline.traffic` comes from the committed counter summary: one entry
    per tiling, valid only for the kernel sources it was taken on."""
    b = _bench_module()
    sha = b.source_hash(b.KERNEL_SOURCES["fgp_fused"])
    (tmp_path / "hbm_traffic_fgp_fused_cacti_1024x24.txt").write_text(
        "# comment: not a key\n"
        f"kernel_source_sha256: {sha}\n"
        "hbm_bytes_per_launch[shape9/passes1]: 201751461\n"
        "hbm_bytes_per_launch[shape7/passes1]: 201761697\n")
    b.PROFILE_DIR = str(tmp_path)
    assert b.read_traffic("fgp_fused", "shape9/passes1") == 201751461.0
    assert b.read_traffic("fgp_fused", "shape7/passes1") == 201761697.0
    assert b.read_traffic("fgp_fused", "shape3/passes2") is None
    (tmp_path / "hbm_traffic_fgp_fused_cacti_1024x24.txt").write_text(
        "kernel_source_sha256: 0000000000000000\nhbm_bytes_per_launch[shape9/passes1]: 1\n")
    assert b.read_traffic("fgp_fused", "shape9/passes1") is None
    assert b.read_traffic("fgp_stream", "stream") is None  # no summary for this family
