"""bench.py's output contract: one JSON line with the fields the benchmark
record needs (metric, value, unit, n_gpus, steps, warmup, ms_per_step,
higher_is_better, scaling, vs_baseline, dtype, data, config, roofline,
cpu_baseline), and a refusal of more than one GPU."""
import json
import sys

import pytest


def test_bench_refuses_several_gpus(monkeypatch, capsys):
    import bench
    monkeypatch.setattr(sys, "argv", ["bench.py", "--gpus", "2"])
    with pytest.raises(SystemExit) as e:
        bench.main()
    assert e.value.code == 2
    assert "one GPU" in capsys.readouterr().err


@pytest.mark.gpu
def test_bench_line_fields(monkeypatch, capsys):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    import bench
    monkeypatch.setattr(sys, "argv", ["bench.py", "--steps", "8", "--warmup", "4", "--n-fluid", "100000",
                                      "--no-surrogate", "--no-batch", "--no-cpu-baseline", "--quiet"])
    bench.main()
    lines = [ln for ln in capsys.readouterr().out.splitlines() if ln.startswith("{")]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 8 and d["warmup"] == 4 and d["higher_is_better"] is True
    assert d["value"] > 0 and d["ms_per_step"] > 0 and d["vs_baseline"] is None and d["cpu_baseline"] is None
    assert d["unit"] == "particle-updates/s" and "workload" in d["config"]
    r = d["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in r, k
    assert 0 < r["frac"] < 1 and r["achieved"] == pytest.approx(r["frac"] * r["peak"], rel=1e-3)


def test_cpu_baseline_protocol(monkeypatch):
    """The CPU-baseline record: the oracle timed on all threads and on one
    thread, with the CPU model, and the FP64 dam break beside it (here on
    small stand-in scenes so the test stays short)."""
    import bench
    from paper_2511_15908_amd import scenes
    small = scenes.small_scene(seed=41, nf=(5, 4, 4), n_tank=(10, 8, 8))
    monkeypatch.setattr(scenes, "dam_break", lambda: scenes.small_scene(seed=42, nf=(4, 4, 4), n_tank=(8, 6, 6),
                                                                        precision="f64"))
    r = bench.cpu_baseline(small)
    assert r["kind"] == "oracle" and r["unit"] == "particle-updates/s" and r["cores"] >= 1
    assert r["value"] > 0 and r["one_thread"]["value"] > 0 and isinstance(r["cpu_model"], str)
    assert r["dam_break_fp64"]["all_threads"]["steps"] == 100 and r["dam_break_fp64"]["one_thread"]["steps"] == 10
    assert "3 full FP64 oracle steps" in r["sample"]
