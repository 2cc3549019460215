"""The learned wrench surrogate end to end on the GPU: plain-SPH haptic logs
of the 100k-particle haptic scene (a 1 kHz hand-like walk of the grabbed
sphere, 4 SPH steps per tick, 40 ms haptic rolling mean), training by the
library's own forward/backward/Adam kernels, and the gain over the haptic
loop without the network (zero-order hold of the 100 Hz SPH wrench, and the
hold followed by a rolling mean) on three walks it never saw, judged against
plain SPH at every tick."""
import pytest

pytestmark = pytest.mark.gpu


def test_surrogate_beats_hold_between_sph_updates():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2511_15908_amd import surrogate as S
    r = S.run_experiment(train_segments=4, ticks=3000, eval_ticks=1500, steps=1500,
                         log=lambda m: print(m, flush=True))
    e = r["errors"]
    print({k: round(v["mean"], 4) for k, v in e.items()}, "p95",
          {k: round(v["p95"], 4) for k, v in e.items()},
          f"rates {r['host_round_trip_hz']:.0f} Hz host, {r['device_chain_hz']:.0f} Hz device")
    # pooled over three evaluation walks; the hold's error swings several-fold
    # with a walk's smoothness, the surrogate's much less: it must beat both
    # baselines on the mean and the hold clearly on the tail
    base = min(e["zero_order_hold"]["mean"], e["hold_rolling_mean"]["mean"])
    assert e["surrogate"]["mean"] < base
    assert e["surrogate"]["p95"] < 0.85 * e["zero_order_hold"]["p95"]
    assert r["host_round_trip_hz"] > 1000.0
