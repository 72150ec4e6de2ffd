"""Parity of the reaction-rate-equation sweep (rn_ode_sweep) with the FP64
oracle, for both integrators: the Dormand-Prince 5(4) pair and the Rosenbrock
4(3) method for stiff networks.

Both sides evaluate the same stage formulas in the same order without fused
multiply-adds (for the Rosenbrock method also the Jacobian, the pivoted LU
factorization and the triangular solves); only the step-size factor
err^(-1/5) or err^(-1/4) goes through pow(), whose host and device versions may
differ in the last bit, and the device sums the error norm over species in a
butterfly order.  A different last bit in a step size moves the solution by
about rtol * |y| at most, so samples are compared within 10 * rtol * (1 + |y|),
each trajectory's step total within 5%, the sweep's within 0.5%, and status
bits must be equal."""
import numpy as np
import pytest

import oracle
from paper_1309_7695_amd import gen, rn

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _check(w, rtol=1e-6, atol=1e-6, method="dopri5"):
    print(f"case ode {method} {w.name}: T={w.n_traj} rtol={rtol}", flush=True)
    out, st = rn.ode_run(w.net, w.rates, w.x0, w.times, rtol=rtol, atol=atol, method=method)
    ref, rst = oracle.ode_run(w.net, w.rates, w.x0, w.times, rtol=rtol, atol=atol, threads=8,
                              method=method)
    err = np.abs(out - ref) / (1.0 + np.abs(ref))
    same_steps = np.all(st == rst, axis=1).mean()
    tot = st[:, :2].sum(axis=1).astype(float)
    rtot = rst[:, :2].sum(axis=1).astype(float)
    rel = np.abs(tot - rtot) / rtot
    agg = abs(tot.sum() / rtot.sum() - 1.0)
    print(f"  max rel diff {err.max():.3g}, identical step counts {same_steps:.4f}, "
          f"max step-total diff {rel.max():.3g}, aggregate {agg:.3g}", flush=True)
    assert np.all(st[:, 3] == rst[:, 3])
    samp, steps, total = TOL[method]
    assert err.max() <= samp * rtol
    assert rel.max() <= steps
    assert agg <= total
    return out, st


# (samples in rtol * (1 + |y|), one trajectory's step total, the sweep's step
# total).  Dormand-Prince: from the oracle with its pow nudged by one ulp.
# Rosenbrock: from the oracle with its pow nudged by one ulp either way and its
# error-norm sums taken in the device's butterfly order, which moved samples by
# up to 15.3 rtol (stiff network, rtol 1e-8), a short trajectory's step total
# (164 steps) by 16.7% and a sweep's total by 3.6e-4.
TOL = {"dopri5": (10.0, 0.05, 0.005), "ros4": (25.0, 0.25, 0.001)}


def test_ode_enzyme():
    _check(gen.enzyme_workload())


def test_ode_synthetic_ragged():
    _check(gen.synthetic_workload(n_traj=300, t_end=5.0, n_samples=21))


def test_ode_stiff_subset_tight_tolerance():
    _check(gen.stiff_workload(n_traj=70), rtol=1e-8, atol=1e-8)


def test_ode_closed_form_decay_on_gpu():
    net = gen.decay_network()
    rates = np.full((1, 130), 0.7)
    times = gen.sample_times(5.0, 11)
    out, st = rn.ode_run(net, rates, np.array([1000], np.int32), times, rtol=1e-10, atol=1e-10)
    assert np.allclose(out[:, 0, :], (1000 * np.exp(-0.7 * times))[:, None], rtol=1e-8)


def test_ode_wide_network_lane_kernel():
    # more than 64 species: the lane-per-trajectory kernel with its workspace
    _check(gen.synthetic_workload(n_traj=130, n_species=70, n_reactions=140, t_end=1.0,
                                  n_samples=6, seed=3))


def test_ode_full_size_sample():
    # the benchmark's rate-equation sweep at full size (65,536 trajectories, the
    # 50x100 workload to t_end 50); 8 spread trajectories re-run by the oracle
    w = gen.synthetic_workload()
    print(f"case ode full size: T={w.n_traj}", flush=True)
    out, st = rn.ode_run(w.net, w.rates, w.x0, w.times)
    ids = np.linspace(0, w.n_traj - 1, 8).astype(int)
    for t in ids:
        ref, rst = oracle.ode_run(w.net, w.rates, w.x0, w.times, traj_range=(int(t), int(t) + 1))
        err = (np.abs(out[:, :, t] - ref[:, :, 0]) / (1.0 + np.abs(ref[:, :, 0]))).max()
        tot, rtot = float(st[t, :2].sum()), float(rst[0, :2].sum())
        assert err <= 10 * 1e-6, (t, err)
        assert abs(tot - rtot) / rtot <= 0.05, (t, tot, rtot)
        assert st[t, 3] == rst[0, 3]
    print("  8 sampled trajectories within the rate-equation tolerance", flush=True)


@pytest.mark.parametrize("n_species,n_reactions", [(64, 128), (64, 160), (40, 200)])
def test_ode_wave_kernel_boundaries(n_species, n_reactions):
    # the wave kernel at its edges: 64 species (lane 63 owns a species and the
    # pseudo-species sits past the wave), and reactions past the two register
    # slots of a lane (j >= 128: rates from LDS, laws from the tables)
    _check(gen.synthetic_workload(n_traj=150, n_species=n_species, n_reactions=n_reactions,
                                  t_end=1.0, n_samples=6, seed=31))


# The Rosenbrock 4(3) method (RN_ODE_ROS4), the stiff integrator.

def test_ros4_stiff_subset():
    # the stiff 30x80 network (rates over eight decades): the oracle's explicit
    # pair needs ~1e5 steps per trajectory here, the Rosenbrock method ~1e3
    _check(gen.stiff_workload(n_traj=300), method="ros4")


def test_ros4_stiff_tight_tolerance():
    _check(gen.stiff_workload(n_traj=70), rtol=1e-8, atol=1e-8, method="ros4")


def test_ros4_enzyme():
    _check(gen.enzyme_workload(), method="ros4")


def test_ros4_synthetic_ragged():
    _check(gen.synthetic_workload(n_traj=200, t_end=5.0, n_samples=21), method="ros4")


@pytest.mark.parametrize("n_species,n_reactions", [(64, 128), (64, 160), (40, 200), (1, 2)])
def test_ros4_boundaries(n_species, n_reactions):
    # 64 species (every lane a row of W), reactions past the two register
    # slots of a lane, and a single species
    _check(gen.synthetic_workload(n_traj=90, n_species=n_species, n_reactions=n_reactions,
                                  t_end=1.0, n_samples=6, seed=31), method="ros4")


def test_ros4_closed_form_decay():
    net = gen.decay_network()
    rates = np.full((1, 70), 0.7)
    times = gen.sample_times(5.0, 11)
    out, st = rn.ode_run(net, rates, np.array([1000], np.int32), times, rtol=1e-10, atol=1e-10,
                         method="ros4")
    assert np.allclose(out[:, 0, :], (1000 * np.exp(-0.7 * times))[:, None], rtol=1e-7)


def test_ros4_refuses_networks_beyond_a_wave():
    w = gen.synthetic_workload(n_traj=4, n_species=70, n_reactions=140, t_end=1.0, n_samples=3)
    with pytest.raises(rn.RNError) as e:
        rn.ode_run(w.net, w.rates, w.x0, w.times, method="ros4")
    assert e.value.code == rn.RN_E_UNSUPPORTED


def test_ros4_stiff_full_size_sample():
    # the stiff configuration at its stated size (65,536 trajectories, t_end
    # 10): 8 spread trajectories re-run by the oracle
    w = gen.stiff_workload()
    print(f"case ros4 stiff full size: T={w.n_traj}", flush=True)
    out, st = rn.ode_run(w.net, w.rates, w.x0, w.times, method="ros4")
    assert np.all(st[:, 3] == 0)
    ids = np.linspace(0, w.n_traj - 1, 8).astype(int)
    for t in ids:
        ref, rst = oracle.ode_run(w.net, w.rates, w.x0, w.times, traj_range=(int(t), int(t) + 1),
                                  method="ros4")
        err = (np.abs(out[:, :, t] - ref[:, :, 0]) / (1.0 + np.abs(ref[:, :, 0]))).max()
        tot, rtot = float(st[t, :2].sum()), float(rst[0, :2].sum())
        assert err <= TOL["ros4"][0] * 1e-6, (t, err)
        assert abs(tot - rtot) / rtot <= TOL["ros4"][1], (t, tot, rtot)
    print(f"  8 sampled trajectories within the rate-equation tolerance; accepted steps "
          f"mean {st[:, 0].mean():.0f} max {st[:, 0].max()}", flush=True)
