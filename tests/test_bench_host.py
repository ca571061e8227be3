"""Host-side logic of bench.py (no GPU): the algorithmic flop and byte models
behind the roofline entry, the choice of the bound, the counter-traffic
lookup and the single-GPU guard."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_flop_model_at_d100():
    f = bench.kernel_flops("fp32", 100, 110, 2, 32, 4096)
    rows = 4096 * 31
    # d -> w, w -> w, w -> d products, two flops per multiply-add
    assert f["forward"] == 2 * (110 * 100 + 110 * 110 + 100 * 110) * rows == 68_200 * rows
    # the reverse sweep has no input gradient at the first layer
    assert f["backward"] == 2 * (110 * 100 + 110 * 110) * rows
    # weight gradients: same products plus one add per bias, plus dZ0
    assert f["wgrad"] == (68_200 + 2 * 110 + 100) * rows + 100 * 4096


def test_byte_model_at_d100():
    b32 = bench.kernel_alg_bytes("fp32", 100, 110, 2, 32, 4096)
    b16 = bench.kernel_alg_bytes("bf16", 100, 110, 2, 32, 4096)
    rows = 4096 * 31
    nw = 31 * (110 * 101 + 110 * 111 + 100 * 111)   # weights and biases of the 31 step networks
    # weights once in the GEMM precision and two fp32 scalars per path-step
    assert b32["forward"] == 4 * nw + 8 * rows
    assert b16["forward"] == 2 * nw + 8 * rows
    # the weight gradient is written once in fp32 whatever the GEMM precision
    assert b16["wgrad"] == b32["wgrad"] == 4 * nw + 8 * rows


def test_roofline_uses_the_matrix_peak_of_the_dtype():
    kern = {"forward": 0.10, "backward": 0.08, "wgrad": 0.12}
    dom, r = bench.roofline_entry("fp32", kern)
    assert dom == "wgrad"
    assert r["bound"] == "mfma" and r["unit"] == "TFLOP/s" and r["peak"] == 157.3
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"], rel=1e-3)
    flops = bench.kernel_flops("fp32", 100, 110, 2, 32, 4096)["wgrad"]
    assert r["achieved"] == pytest.approx(flops / 0.12e-3 / 1e12, rel=1e-3)
    dom, r = bench.roofline_entry("bf16", kern)
    assert r["bound"] == "mfma" and r["peak"] == 2500.0
    flops = bench.kernel_flops("bf16", 100, 110, 2, 32, 4096)["wgrad"]
    assert r["frac"] == pytest.approx(flops / 0.12e-3 / 1e12 / 2500.0, rel=1e-3)
    # intensity on the algorithmic byte basis is far above both ridge points
    nbytes = bench.kernel_alg_bytes("bf16", 100, 110, 2, 32, 4096)["wgrad"]
    assert flops / nbytes > 2500.0 / 8.0
    assert r["algorithmic_bytes"] == nbytes


def test_roofline_of_the_fused_reverse_kernel():
    """The fused reverse kernel is timed in the backward slot with no
    weight-gradient launches: it is reported as "reverse" and carries the
    flops of both the reverse sweep and the weight gradient."""
    kern = {"forward": 0.10, "backward": 0.19, "wgrad": 0.0, "reduce": 0.01}
    dom, r = bench.roofline_entry("fp32", kern)
    assert dom == "reverse"
    f = bench.kernel_flops("fp32", 100, 110, 2, 32, 4096)
    assert f["reverse"] == f["backward"] + f["wgrad"]
    assert r["achieved"] == pytest.approx(f["reverse"] / 0.19e-3 / 1e12, rel=1e-3)
    # the separate pair is untouched
    assert bench.reverse_kernels({"forward": 0.1, "backward": 0.08, "wgrad": 0.12}) == \
        {"forward": 0.1, "backward": 0.08, "wgrad": 0.12}


def test_step_quantiles():
    q = bench._quantiles([1.0, 2.0, 3.0, 4.0, 5.0, 6.0, 7.0, 8.0, 9.0, 10.0])
    assert q["n"] == 10 and q["median"] == 5.5 and q["p10"] == pytest.approx(1.9) and q["p90"] == pytest.approx(9.1)


def test_traffic_lookup_requires_the_profiled_source(tmp_path, monkeypatch):
    rec = json.load(open(os.path.join(ROOT, "profiles", "bsb_d100_traffic.json")))
    t = bench.measured_traffic("reverse", "fp32")
    src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    import hashlib
    if hashlib.sha256(src).hexdigest() == rec["source_sha256"]:
        per = rec["per_launch"]["reverse_fp32"]
        assert t == int(round(per["read_bytes"] + per["write_bytes"]))
    else:
        assert t is None
    # a counter file taken on another source gives no traffic figure
    fake = dict(rec, source_sha256="0" * 64)
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "bsb_d100_traffic.json").write_text(json.dumps(fake))
    (tmp_path / os.path.dirname(rec["source"])).mkdir(parents=True)
    (tmp_path / rec["source"]).write_bytes(src)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("wgrad", "fp32") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert "one GPU" in (r.stdout + r.stderr)
