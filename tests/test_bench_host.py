"""Host-side logic of bench.py (no GPU): the one-GPU refusal, the byte models, the
kernel-source hash that keys the committed byte-counter records, and the records
themselves."""
import json
import os
import shutil
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def _bench():
    argv = sys.argv
    sys.argv = ["bench.py"]
    try:
        import bench
    finally:
        sys.argv = argv
    return bench


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_byte_models_by_hand():
    b = _bench()
    # c2: Q=9, d=2, N_g=18,721, N_l=25,088: 8 * (81 N_g + 3 (8 N_l + 4 N_g)) bytes
    assert b.step_model_bytes(9, 2, 18721, 25088) == 8.0 * (81 * 18721 + 3 * (8 * 25088 + 4 * 18721))
    # kernel C of the fused path: ((Q-1) + 1 + Q + 2Q/3 + Q + 2) N_g + d(d+1)/2 N_l doubles
    ng, nl = 1000, 1500
    assert b.algorithmic_bytes("f_rk_lap", 9, 2, ng, nl) == 8.0 * ((8 + 1 + 9 + 6 + 9 + 2) * ng + 3 * nl)
    # node kernel rk: Q-1 partials per local copy, then Q + 2Q/3 + 1 + Q + 1 doubles per node
    assert b.algorithmic_bytes("rk", 19, 3, ng, nl) == 8.0 * (18 * nl + (19 + 38 / 3.0 + 1 + 19 + 1) * ng)
    # with ni element-interior nodes finished by the element kernels, rk covers the others
    ni = 300
    assert b.algorithmic_bytes("rk", 19, 3, ng, nl, ni) == \
        8.0 * (18 * (nl - ni) + (19 + 38 / 3.0 + 1 + 19 + 1) * (ng - ni))
    # ... and the streaming kernel finishes the interior nodes: + (1 + 2Q/3 + 1 + Q + 1) each
    assert b.algorithmic_bytes("stream", 19, 3, ng, nl, ni) == \
        8.0 * (18 * ng + 2 * ng + 9 * nl + (1 + 38 / 3.0 + 1 + 19 + 1) * ni + 18 * (nl - ni))


def test_kernel_hash_ignores_comments_but_not_code(tmp_path):
    b = _bench()
    src = os.path.join(ROOT, "paper_2609_00535_amd", "csrc")
    dst = tmp_path / "csrc"
    shutil.copytree(src, dst)
    h0 = b.kernels_sha256(str(dst))
    assert h0 == b.kernels_sha256(src)
    k = dst / "kernels.hpp"
    text = k.read_text()
    k.write_text("// a comment line\n\n" + text.replace("\n", "\n// another\n", 1))
    assert b.kernels_sha256(str(dst)) == h0
    k.write_text(text + "\nconstexpr int kUnused = 1;\n")
    assert b.kernels_sha256(str(dst)) != h0


def test_committed_traffic_records_match_the_kernels():
    """bench.py reports the committed byte counts only while they were taken on the
    current kernel source; records of older kernels are skipped here and reported as
    null by bench.py."""
    import pytest
    b = _bench()
    for w, kind in (("c2", "f_rk_lap"), ("c3", "f_rk_lap"), ("c2xl", "stream"), ("c4", "rk")):
        rec = json.load(open(os.path.join(ROOT, "profiles", f"traffic_{w}.json")))
        if rec["kernels_sha256"] != b.kernels_sha256():
            assert b.traffic_from_profiles(w, kind) is None
            pytest.skip(f"traffic_{w}.json predates the current kernels")
        assert b.traffic_from_profiles(w, kind) == float(rec["bytes_per_launch"][kind])
        cal = rec["calibration"]
        assert abs(cal["fetch_scale"] - 2.0) < 1e-3 and abs(cal["write_scale"] - 1.0) < 1e-3
    assert b.traffic_from_profiles("no_such_workload", "rk") is None


def test_fp64_rate_from_counted_flops():
    """The step's FP64 rate: each kind's flops per launch times its launches per profiled
    step, over the step time; null when a kind in the step has no count."""
    b = _bench()
    flops = {"stream": 6.0e9, "rk": 1.0e9, "lap": 5.0e8}
    # (ms over the profiled steps, launches over the profiled steps), 2 profiled steps
    prof = {"stream": (3.0, 6), "rk": (1.5, 6), "lap": (0.5, 6)}
    r = b.fp64_point(flops, prof, 2, 2.5, "stream", 0.5, 4.0e9)
    per_step = 3 * 6.0e9 + 3 * 1.0e9 + 3 * 5.0e8
    assert abs(r["flops_per_step"] - per_step) < 1.0
    assert abs(r["achieved"] - per_step / 2.5e-3 / 1e12) < 1e-9
    assert abs(r["frac"] - r["achieved"] / 78.6) < 1e-12 and r["unit"] == "TFLOP/s"
    assert abs(r["kernel_achieved"] - 6.0e9 / 0.5e-3 / 1e12) < 1e-9
    assert abs(r["flop_per_model_byte"] - per_step / 4.0e9) < 1e-12
    assert b.fp64_point({"stream": 1.0}, prof, 2, 2.5, "stream", 0.5, 4.0e9) is None
    assert b.fp64_point(None, prof, 2, 2.5, "stream", 0.5, 4.0e9) is None


def test_committed_fp64_records_match_the_kernels():
    """The committed FP64 instruction counts: taken on the current kernels (else skipped
    and reported as null), flops = 64 x (add + mul + trans + 2 fma) per launch."""
    import pytest
    b = _bench()
    for w in ("c2", "c3", "c2xl", "c4", "c4q13"):
        rec = json.load(open(os.path.join(ROOT, "profiles", f"fp64_{w}.json")))
        if rec["kernels_sha256"] != b.kernels_sha256():
            assert b.fp64_from_profiles(w) is None
            pytest.skip(f"fp64_{w}.json predates the current kernels")
        got = b.fp64_from_profiles(w)
        for kind, n in rec["instructions_per_launch"].items():
            f = 64 * (n["VALU_ADD_F64"] + n["VALU_MUL_F64"] + n["VALU_TRANS_F64"] + 2 * n["VALU_FMA_F64"]) \
                + 512 * n["VALU_MFMA_MOPS_F64"]
            assert abs(got[kind] - f) <= 1e-9 * f
            assert n["VALU_MFMA_MOPS_F64"] == 0.0  # vector FP64 only
    assert b.fp64_from_profiles("no_such_workload") is None
