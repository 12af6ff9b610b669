"""Host-side parts of bench.py: the one-GPU contract, the algorithmic work
model and the staleness hash of the step kernels' sources."""
import os
import subprocess
import sys

import bench
from workloads import make_workload

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_work_model_scales_with_elements():
    a = make_workload("c2", n=3, N=3)
    b = make_workload("c2", n=6, N=3)
    fa, fb = bench.flops_per_launch(a), bench.flops_per_launch(b)
    ba, bb = bench.bytes_per_launch(a, "fp32"), bench.bytes_per_launch(b, "fp32")
    for k in ("predict", "volume", "lift_update"):      # element kernels (faces: boundary share)
        assert fb[k] == 8 * fa[k] and bb[k] == 8 * ba[k]
    # about 401 kFLOP per element for the prediction and volume terms at degree 3
    assert abs((fa["predict"] + fa["volume"]) / a.ne - 401120) < 1.0
    # FP64 states move more bytes than FP32 ones
    assert bench.bytes_per_launch(a, "fp64")["predict"] > ba["predict"]


def test_source_hash_ignores_comments(tmp_path, monkeypatch):
    csrc = os.path.join(ROOT, "paper_2502_09714_amd", "csrc")
    h0 = bench.kernel_source_hash()
    root = tmp_path / "r"
    (root / "paper_2502_09714_amd" / "csrc").mkdir(parents=True)
    for f in bench.HASHED_SOURCES:
        src = open(os.path.join(csrc, f)).read()
        if f == "mfma.hpp":
            src = "// an added comment\n/* and a block\n   comment */\n" + src.replace("\n", "  // note\n", 3)
        (root / "paper_2502_09714_amd" / "csrc" / f).write_text(src)
    build = open(os.path.join(ROOT, "paper_2502_09714_amd", "build.py")).read()
    (root / "paper_2502_09714_amd" / "build.py").write_text(build)
    monkeypatch.setattr(bench, "ROOT", str(root))
    assert bench.kernel_source_hash() == h0
    # a code change in the launch code, or another compiler flag, changes it
    p = root / "paper_2502_09714_amd" / "csrc" / "dgd.hip"
    p.write_text(p.read_text() + "\nint x;\n")
    assert bench.kernel_source_hash() != h0
    p.write_text(open(os.path.join(csrc, "dgd.hip")).read())
    assert bench.kernel_source_hash() == h0
    (root / "paper_2502_09714_amd" / "build.py").write_text(build.replace('"-O3"', '"-O2"'))
    assert bench.kernel_source_hash() != h0
