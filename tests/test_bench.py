"""Host-side contract of bench.py: the one-GPU exit, the counter summary it reads only while the kernels are
unchanged, the full-vector error metric, and its CPU oracle legs (workload and gradient) on small grids."""
import json
import os
import subprocess
import sys

import numpy as np

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    lines = [ln for ln in r.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1
    msg = json.loads(lines[0])
    assert "one GPU" in msg["error"] and msg["n_gpus"] == 2


def test_traffic_summary_used_only_for_current_kernels(tmp_path, monkeypatch):
    # a summary taken on other sources is ignored; one taken on the current sources is read
    f = tmp_path / "t.txt"
    f.write_text("sources_sha256_16: 0000000000000000\nhbm_bytes_per_step: 123.0\n")
    monkeypatch.setattr(bench, "TRAFFIC", str(f))
    assert bench.traffic_per_step() is None
    f.write_text(f"sources_sha256_16: {bench.sources_sha16()}\nhbm_bytes_per_step: 123.0\n")
    assert bench.traffic_per_step() == 123.0
    if os.path.exists(os.path.join(ROOT, "profiles", "stage_solve_traffic.txt")):
        vals = dict(ln.split(":", 1) for ln in open(os.path.join(ROOT, "profiles", "stage_solve_traffic.txt"))
                    if ":" in ln)
        assert float(vals["hbm_bytes_per_step"]) > 0


def test_error_metric_is_the_whole_vector_at_every_step():
    ref = [np.ones(10) * (k + 1) for k in range(3)]
    states = [r.copy() for r in ref]
    states[1][4] += 2e-3 * np.linalg.norm(ref[1])
    e = bench.rel_errors(states, ref)
    assert e["steps_compared"] == 3 and e["rel_l2_final"] == 0.0
    assert abs(e["rel_l2_max_over_steps"] - 2e-3) < 1e-12
    assert bench.rel_errors([], ref) is None and bench.rel_errors(states, None) is None


def test_oracle_tier_needs_a_diagonalisable_tableau():
    assert bench.distinct_eigenvalues([[0.2, 0.0], [0.3, 0.4]])
    assert not bench.distinct_eigenvalues([[0.4, 0.0], [0.3, 0.4]])


def test_cpu_leg_on_a_small_grid():
    args = bench.parse(["--N", "16", "--steps", "3"])
    leg = bench.cpu_leg(args, want_config2=False, want_config3=False)
    cb = leg["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["cores"] == 1 and cb["value"] > 0
    assert cb["host"]["nproc"] >= 1
    refs = leg["refs"]["main"]
    assert len(refs) == 3 and refs[0].shape == (15 * 15,)
    # the solution decays (heat equation, zero Dirichlet data)
    assert np.linalg.norm(refs[-1]) < np.linalg.norm(refs[0])


def test_cpu_leg_adjoint_compares_whole_vectors():
    # the oracle's coupled-LU gradient on a small grid, handed in as if it came from the GPU: the CPU leg's
    # decoupled-tier gradient agrees to rounding; a perturbation of one element shows up as its relative size
    from oracle import adjoint, step
    from oracle import tableaux as T
    import synth

    N, steps, dt = 16, 3, 1e-3
    tab = T.radau_iia(3)
    kap = synth.grf_kappa(N, 1)
    u0, _ = synth.sine_modes_u0(N, 0)
    ustar = step.run(N, synth.grf_kappa(N, 2), tab, dt, steps, u0)[-1]
    fwd = adjoint.forward(N, kap, tab, dt, steps, u0)
    J, lamN = adjoint.objective(fwd[2], fwd[0][-1], ustar)
    lam0, g = adjoint.gradient(N, kap, tab, dt, steps, u0, lamN, fwd=fwd)
    e = bench.cpu_leg_adjoint(g, lam0, J, N=N, steps=steps, dt=dt)
    assert e["grad_rel_l2"] < 1e-10 and e["lam0_rel_l2"] < 1e-10 and e["J_rel"] < 1e-10
    g2 = g.copy()
    g2[7] += 1e-3 * np.linalg.norm(g)
    assert abs(bench.cpu_leg_adjoint(g2, lam0, J, N=N, steps=steps, dt=dt)["grad_rel_l2"] - 1e-3) < 1e-6
