"""CPU checks of bench.py's command line: more than one GPU is refused with
a message (this library has no multi-GPU path), and the kernel-source hash
that gates the stored HBM-traffic figure ignores comments only."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr and p.stdout == ""


def test_kernel_source_hash_ignores_comments(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench

    h = bench.kernel_source_hash()
    csrc = tmp_path / "paper_2412_16370_amd" / "csrc"
    csrc.mkdir(parents=True)
    srcs = {}
    for name in ("ppc_device.hpp", "ppc_plain.hip"):
        with open(os.path.join(ROOT, "paper_2412_16370_amd", "csrc", name)) as f:
            srcs[name] = f.read()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    # comments and blank lines added: same hash
    (csrc / "ppc_device.hpp").write_text("// a new comment\n\n/* and a block\n comment */\n" + srcs["ppc_device.hpp"])
    (csrc / "ppc_plain.hip").write_text(srcs["ppc_plain.hip"] + "\n// trailing comment\n")
    assert bench.kernel_source_hash() == h
    # one token of code changed: another hash
    (csrc / "ppc_plain.hip").write_text(srcs["ppc_plain.hip"].replace("kMaxTilesPerWave = 1ull << 20",
                                                                     "kMaxTilesPerWave = 1ull << 19"))
    assert bench.kernel_source_hash() != h
