"""The host-only parts of bench.py run on the CPU: the oracle's bounded
cpu_baseline sample (on a small box, so that the suite stays quick) returns a
positive rate with its sample description, and the workload draws of the
batch and warm-start studies are reproducible."""
import math

from workloads import config, batch_draws, parameter_draws


def test_cpu_baseline_runs_on_a_small_box():
    import bench
    r = bench.cpu_baseline(config("small_4x4"))
    assert r["kind"] == "oracle" and r["value"] > 0 and math.isfinite(r["value"])
    assert r["cores"] >= 1 and "BSE blocks" in r["sample"]
    assert set(r["stage_seconds"]) == {"single_particle", "bse", "remap", "sigma_tilde2", "sigma_box"}


def test_study_draws_are_seeded():
    a, b = batch_draws(64, 4), batch_draws(64, 4)
    assert a == b and len({p.Nv for p in a}) == 4
    assert all(0.5 <= p.U <= 3 and 2 <= p.beta <= 8 and 0.8 <= p.filling <= 1 and p.mu_mode == 1 for p in a)
    box = {"U": (1.0, 2.0), "tp": (-0.2, 0.0)}
    x = parameter_draws(config("c2"), box, range(5))
    assert x == parameter_draws(config("c2"), box, range(5))
    assert all(1.0 <= p.U <= 2.0 and -0.2 <= p.tp <= 0.0 for p in x)
