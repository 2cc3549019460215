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
