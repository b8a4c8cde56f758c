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


def test_update_launch_model():
    """The launch model behind the update kernel's roofline: pairing panels
    changes the launches, not the work, so the multiply-adds of the modelled
    launches equal the sum over single panels (forward: rows below x columns
    right of the panel, A and B; back substitution: rows above x the n columns
    of B); with n = 1024 a solve makes 20 launches."""
    import bench

    for n in (256, 384, 512, 1024):
        L = bench.update_launches(n)
        macs = sum(r * c * k for r, c, k, m in L)
        fwd = sum((n - 128 * (j + 1)) * ((n - 128 * (j + 1)) + n) * 128 for j in range(n // 128))
        back = sum(128 * j * n * 128 for j in range(n // 128))
        assert macs == fwd + back, n
        assert sum(m for r, c, k, m in L) == n - 128          # every row but the last panel's is mixed here
    assert len(bench.update_launches(1024)) == 20

    class D:
        n, Nq = 1024, 960
    c = bench.update_compulsory(D)
    assert c["launches"] == 20 and c["flops"] == 8.0 * (fwd + back) * 960 / 20     # fwd, back of n = 1024
