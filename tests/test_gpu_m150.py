"""GPU parity on the 150-species mechanism (N = 151): the block kernel (one
512-lane block per state, FP32 factors with FP64 refinement) and the
lane-per-state kernel (slow: matrices in global memory, so its batches are
small).  Same bar as the other mechanisms: max relative error <= 1e-5 on T
and on every Y_i whose oracle value exceeds 1e-8."""
import numpy as np
import pytest

from paper_1607_03884_amd import configs, gen
from tests.parity import banner, integration_errors, rhs_magnitudes, EPS

pytestmark = pytest.mark.gpu

K = 150


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def m150_path():
    return configs.mech_path("M150")


@pytest.fixture(scope="module")
def g150(torch_dev, m150_path):
    from paper_1607_03884_amd import Mechanism
    return Mechanism(m150_path)


@pytest.fixture(scope="module")
def o150(oracle_mod, m150_path):
    return oracle_mod.Mech(m150_path)


def _dev(torch_dev, rows):
    torch, dev = torch_dev
    return torch.from_numpy(gen.to_soa(rows)).to(dev)


def test_m150_rhs_jacobian(torch_dev, g150, o150):
    banner("M150 source terms and Jacobian")
    mech = gen.make_mechanism(configs.MECHS["M150"])
    rows = configs.states_for(configs.WORKLOADS["cfg4"], 24)
    y = _dev(torch_dev, rows)
    f = g150.dbg_rhs(y).cpu().numpy().T
    J = g150.dbg_jacobian(y).cpu().numpy().T.reshape(len(rows), K + 1, K + 1)
    worst = 0.0
    for row, fg, Jg in zip(rows, f, J):
        fr = o150.rhs(row[:K + 1], row[-1])
        mag = rhs_magnitudes(mech, o150, row)
        assert np.all(np.abs(fg - fr) <= 2000 * EPS * mag + 1e-300)
        Jr = o150.jac(row[:K + 1], row[-1])
        scale = np.abs(Jr).max(axis=1, keepdims=True) + 1e-300
        worst = max(worst, float((np.abs(Jg - Jr) / scale).max()))
    assert worst <= 1e-11, worst


@pytest.mark.parametrize("dt", [1e-6, 1e-4])
def test_m150_lane_parity(torch_dev, g150, o150, dt):
    """The first five PaSR-like M150 states (burnt ones, 25-55 steps each) over
    each global step, lane kernel.  The lane kernel keeps its N x N matrices
    in global memory, so each elimination step waits on memory: a state
    costs seconds, which bounds the batch of this test."""
    torch, _ = torch_dev
    banner(f"M150 cfg4 5 states dt={dt} lane")
    rows = configs.states_for(configs.WORKLOADS["cfg4"], 5)
    g150.set_option("variant", "lane")
    out = g150.integrate(_dev(torch_dev, rows), dt, configs.ATOL, configs.RTOL)
    torch.cuda.synchronize()
    st = g150.stats(per_state=True)
    got = out.cpu().numpy().T
    ref, res = o150.integrate(rows, dt)
    assert np.all(res["status"] == 0) and np.all(st["per_state_status"] == 0)
    eT, eY = integration_errors(got, ref, K)
    same = np.mean(st["per_state_steps"] == res["nstep"])
    print(f"M150 lane: kernel {st['kernel_ms']:.1f} ms, steps/state {st['steps'] / len(rows):.1f}, "
          f"max rel err T {eT:.2e} Y {eY:.2e}, identical step counts {same:.4f}")
    assert eT <= 1e-5 and eY <= 1e-5
    assert np.abs(got[:, 1:K + 1].sum(1) - rows[:, 1:K + 1].sum(1)).max() <= 1e-12


@pytest.mark.parametrize("dt", [1e-6, 1e-4])
def test_m150_block_parity(torch_dev, g150, o150, dt):
    """The first 67 PaSR-like M150 states (a ragged count of blocks), block
    kernel, against the oracle; conservation of the mass fractions."""
    torch, _ = torch_dev
    n = 67
    banner(f"M150 cfg4 {n} states dt={dt} block")
    rows = configs.states_for(configs.WORKLOADS["cfg4"], n)
    g150.set_option("variant", "block")
    out = g150.integrate(_dev(torch_dev, rows), dt, configs.ATOL, configs.RTOL)
    torch.cuda.synchronize()
    st = g150.stats(per_state=True)
    got = out.cpu().numpy().T
    ref, res = o150.integrate(rows, dt)
    assert np.all(res["status"] == 0) and np.all(st["per_state_status"] == 0)
    eT, eY = integration_errors(got, ref, K)
    same = np.mean(st["per_state_steps"] == res["nstep"])
    print(f"M150 block: kernel {st['kernel_ms']:.1f} ms, steps/state {st['steps'] / n:.1f} "
          f"(oracle {res['nstep'].mean():.1f}), max rel err T {eT:.2e} Y {eY:.2e}, "
          f"identical step counts {same:.4f}, fp32 fallback {st['fp32_fallback']}")
    assert eT <= 1e-5 and eY <= 1e-5
    assert np.array_equal(got[:, K + 1], rows[:, K + 1])
    # sum Y is conserved to rounding only by exact solves.  The mass and
    # element weights are left null vectors of J, so they are the directions
    # where E = g/h I - J is worst conditioned (cond ~ h ||J|| / g) and the
    # FP32 factors, refined, are least accurate: each step keeps the error of
    # its last Newton solve there, a fraction of the last increment, which
    # the Newton test lets reach O(1) in the error weights (about 1e-7
    # absolute for the major species).  Up to 1e-9 per state at dt = 1e-6;
    # a few 1e-8 on single states at dt = 1e-4 (large steps, cond near 2^24).
    drift = np.abs(got[:, 1:K + 1].sum(1) - rows[:, 1:K + 1].sum(1))
    assert drift.max() <= (1e-8 if dt < 1e-5 else 2e-7), drift.max()
    if dt > 1e-5:
        # the drift is the last increments' solve error: with a tight Newton
        # tolerance (small last increments) it falls to rounding level
        g150.set_option("kappa", "1e-6")
        tight = g150.integrate(_dev(torch_dev, rows), dt, configs.ATOL, configs.RTOL).cpu().numpy().T
        g150.set_option("kappa", "0")
        dt_drift = np.abs(tight[:, 1:K + 1].sum(1) - rows[:, 1:K + 1].sum(1))
        print(f"sum Y drift: default Newton tolerance {drift.max():.2e}, kappa 1e-6 {dt_drift.max():.2e}")
        assert dt_drift.max() <= 1e-10
    g150.set_option("variant", "auto")


def test_m150_block_edges(torch_dev, g150):
    """Empty batch; a non-finite state among good ones (status NONFINITE, its
    row copied, the others unaffected); results identical bit for bit when the
    persistent grid shrinks to a tenth or cost bins reorder the queue (the
    state-to-block mapping changes)."""
    torch, dev = torch_dev
    banner("M150 block edges")
    g150.set_option("variant", "block")
    g150.integrate(torch.zeros((K + 2, 0), dtype=torch.float64, device=dev), 1e-6)
    torch.cuda.synchronize()
    rows = configs.states_for(configs.WORKLOADS["cfg4"], 12)
    bad = rows.copy()
    bad[5, 3] = np.nan
    y = _dev(torch_dev, bad)
    out = g150.integrate(y, 1e-6).cpu().numpy().T
    st = g150.stats(per_state=True)
    assert st["per_state_status"][5] == 3 and np.array_equal(out[5, 4:], bad[5, 4:])
    assert np.all(np.delete(st["per_state_status"], 5) == 0)
    ref = g150.integrate(_dev(torch_dev, rows), 1e-6).cpu().numpy()
    g150.set_option("grid_pct", "10")
    small = g150.integrate(_dev(torch_dev, rows), 1e-6).cpu().numpy()
    g150.set_option("grid_pct", "100")
    assert np.array_equal(ref, small)
    # cost bins reorder the queue, a block may take several states per grab;
    # every state's result stays the same bits
    g150.set_option("binning", "8")
    g150.set_option("tile", "2")
    binned = g150.integrate(_dev(torch_dev, rows), 1e-6).cpu().numpy()
    st = g150.stats()
    assert st["nbins_used"] == 8 and st["tile_used"] == 2
    g150.set_option("binning", "0")
    g150.set_option("tile", "1")
    assert np.array_equal(ref, binned)
    assert np.array_equal(np.delete(out, 5, axis=0), np.delete(ref.T, 5, axis=0))
    g150.set_option("variant", "auto")


def test_m150_group_variants_refused(torch_dev, g150):
    """The wavefront variants refuse N = 151 with an error instead of running."""
    banner("M150 group variants refused")
    from paper_1607_03884_amd._lib import RkError
    rows = configs.states_for(configs.WORKLOADS["cfg4"], 4)
    for v in ("wave", "mixed"):
        g150.set_option("variant", v)
        with pytest.raises(RkError):
            g150.integrate(_dev(torch_dev, rows), 1e-6)
    g150.set_option("variant", "auto")


def test_block_variant_refused_small(torch_dev):
    """The block variant refuses mechanisms with N <= 56 (the wavefront
    kernels own that range) with an error instead of running."""
    banner("block variant refused for M13")
    from paper_1607_03884_amd import Mechanism
    from paper_1607_03884_amd._lib import RkError
    g = Mechanism(configs.mech_path("M13"))
    g.set_option("variant", "block")
    rows = configs.states_for(configs.WORKLOADS["cfg0"], 8)
    with pytest.raises(RkError):
        g.integrate(_dev(torch_dev, rows), 1e-6)
    g.close()


def test_m150_block_autotune(torch_dev, g150):
    """The autotuner runs for the block kernel on a bounded sample (the first
    1024 states) and reports its choice; the tuned call's results equal the
    untuned ones bit for bit."""
    torch, _ = torch_dev
    banner("M150 block autotune")
    rows = configs.states_for(configs.WORKLOADS["cfg4"], 1100)
    g150.set_option("variant", "block")
    ref = g150.integrate(_dev(torch_dev, rows), 1e-6).cpu().numpy()
    g150.set_option("autotune", "1")
    tuned = g150.integrate(_dev(torch_dev, rows), 1e-6).cpu().numpy()
    st = g150.stats()
    g150.set_option("autotune", "0")
    g150.set_option("variant", "auto")
    print(f"block autotune: bins {st['nbins_used']}, grid {st['grid_used']}, tile {st['tile_used']}, "
          f"kernel {st['kernel_ms']:.1f} ms")
    assert st["nbins_used"] in (0, 16) and st["tile_used"] in (1, 2, 4)
    assert np.array_equal(ref, tuned)


def test_m150_block_predicted_bins(torch_dev, g150, o150):
    """The 150-species block form with its queue binned by the network's
    predicted step counts (152-256-256-455, trained on oracle runs): states
    start cold, so every result is bitwise the input-order result, and a
    sample matches the oracle."""
    import os
    from paper_1607_03884_amd import predictor
    path = predictor.path_for("M150", 1e-4)
    if not os.path.exists(path):
        pytest.skip("no M150 predictor file")
    torch, _ = torch_dev
    banner("M150 block predicted-step bins")
    rows = configs.states_for(configs.WORKLOADS["cfg4"], 600)
    g150.set_option("variant", "block")
    ref = g150.integrate(_dev(torch_dev, rows), 1e-4).cpu().numpy()
    s0 = g150.stats(per_state=True)
    g150.set_option("predictor", path)
    g150.set_option("predictor_use", "bins")
    g150.set_option("binning", "16")
    got = g150.integrate(_dev(torch_dev, rows), 1e-4).cpu().numpy()
    st = g150.stats(per_state=True)
    g150.set_option("binning", "0")
    g150.set_option("predictor", "none")
    g150.set_option("predictor_use", "both")
    g150.set_option("variant", "auto")
    print(f"M150 predicted bins: {st['kernel_ms']:.1f} ms vs input order {s0['kernel_ms']:.1f} ms; "
          f"D64 queue order {st['d_mean64_queue']:.3f} vs {st['d_mean64']:.3f}")
    assert st["nbins_used"] == 16 and st["predictor_kept"] == 0
    assert np.array_equal(got, ref)
    # the predicted step counts follow the actual ones (queue order costliest first)
    pick = np.arange(0, 600, 20)
    oref, res = o150.integrate(rows[pick], 1e-4)
    eT, eY = integration_errors(got.T[pick], oref, K)
    assert eT <= 1e-5 and eY <= 1e-5


def test_m150_block_costliest_states(torch_dev, g150, o150):
    """The stiffest states decide parity: the first 8,192 cfg4 states on the
    block kernel, the 2 % costliest (by step count) and a seeded draw against
    the oracle at the acceptance bar."""
    torch, _ = torch_dev
    banner("M150 block costliest states")
    rows = configs.states_for(configs.WORKLOADS["cfg4"], 8192)
    g150.set_option("variant", "block")
    g150.set_option("binning", "16")
    out = g150.integrate(_dev(torch_dev, rows), 1e-4).cpu().numpy().T
    st = g150.stats(per_state=True)
    g150.set_option("binning", "0")
    g150.set_option("variant", "auto")
    steps = st["per_state_steps"]
    pick = np.unique(np.concatenate([np.argsort(steps, kind="stable")[-164:],
                                     np.random.default_rng(11).choice(8192, 64, replace=False)]))
    ref, res = o150.integrate(rows[pick], 1e-4)
    assert np.all(res["status"] == 0) and np.all(st["per_state_status"] == 0)
    eT, eY = integration_errors(out[pick], ref, K)
    same = np.mean(steps[pick] == res["nstep"])
    print(f"M150 costliest: kernel {st['kernel_ms']:.1f} ms, max steps {steps.max()}, "
          f"max rel err T {eT:.2e} Y {eY:.2e}, identical step counts {same:.3f}, fp32_fallback {st['fp32_fallback']}")
    assert eT <= 1e-5 and eY <= 1e-5


def test_m150_block_warm_start(torch_dev, g150, o150):
    """The block kernel started from the 150-species network's predicted first
    step and stage values (kept only when Newton converges on that attempt)
    against the oracle started from the same prediction, which decodes the
    committed predictor file itself; a cold restart for every state whose
    warm attempt fails, as in the oracle."""
    import os
    from oracle import predict as opred
    from paper_1607_03884_amd import predictor
    path = predictor.path_for("M150", 1e-4)
    if not os.path.exists(path):
        pytest.skip("no M150 predictor file")
    torch, _ = torch_dev
    banner("M150 block warm start")
    rows = configs.states_for(configs.WORKLOADS["cfg4"], 192)
    g150.set_option("variant", "block")
    g150.set_option("predictor", path)
    g150.set_option("predictor_use", "both")
    g150.set_option("binning", "16")
    got = g150.integrate(_dev(torch_dev, rows), 1e-4).cpu().numpy().T
    st = g150.stats(per_state=True)
    g150.set_option("binning", "0")
    g150.set_option("predictor", "none")
    g150.set_option("variant", "auto")
    pr = opred.load(path)
    h, z, _ = opred.warm_start(pr, rows, configs.ATOL, configs.RTOL, 1e-4)
    ref, res = o150.integrate_warm(rows, 1e-4, h, z)
    assert np.all(res["status"] == 0) and np.all(st["per_state_status"] == 0)
    eT, eY = integration_errors(got, ref, K)
    same = np.mean(st["per_state_steps"] == res["nstep"])
    kept = int(np.sum(res["warm"] == 1))
    print(f"M150 block warm: kept {st['predictor_kept']} (oracle {kept}), restarted {st['predictor_fallback']}; "
          f"vs same-start oracle T {eT:.2e} Y {eY:.2e}, identical step counts {same:.3f}, "
          f"steps/state {st['steps'] / len(rows):.1f} (oracle {res['nstep'].mean():.1f})")
    assert st["predictor_kept"] + st["predictor_fallback"] == len(rows)
    assert abs(st["predictor_kept"] - kept) <= 2
    assert eT <= 1e-5 and eY <= 1e-5


def test_m150_block_poisoned_predictor(torch_dev, g150, o150, tmp_path):
    """A predictor with garbage outputs (huge stage values, tiny first steps)
    on the block kernel: Newton rejects the predicted stage values, the state
    restarts exactly as a cold start (bitwise the cold result), and every
    result meets the bar against the cold oracle."""
    import os
    from paper_1607_03884_amd import predictor
    torch, _ = torch_dev
    banner("M150 block poisoned predictor")
    N, dt = K + 1, 1e-4
    dims = [K + 2, 16, 3 * N + 2]
    rng = np.random.default_rng(6)
    nparam = sum(dims[i] * dims[i + 1] + dims[i + 1] for i in range(len(dims) - 1))
    params = rng.standard_normal(nparam) * 3.0
    out_shift = np.concatenate([np.full(3 * N, 30.0), [-4.0, 1.0]])
    path = os.path.join(str(tmp_path), "poison150.rkp")
    predictor.write(path, "M150", K, dt, dims, np.zeros(K + 2), np.ones(K + 2), out_shift, np.full(3 * N + 2, 5.0),
                    params)
    rows = configs.states_for(configs.WORKLOADS["cfg4"], 67)
    g150.set_option("variant", "block")
    cold = g150.integrate(_dev(torch_dev, rows), dt).cpu().numpy().T
    g150.set_option("predictor", path)
    g150.set_option("predictor_use", "both")
    got = g150.integrate(_dev(torch_dev, rows), dt).cpu().numpy().T
    st = g150.stats(per_state=True)
    g150.set_option("predictor", "none")
    g150.set_option("variant", "auto")
    ref, res = o150.integrate(rows, dt)
    eT, eY = integration_errors(got, ref, K)
    same = int(np.sum(np.all(got == cold, axis=1)))
    print(f"M150 block poisoned: restarted {st['predictor_fallback']}, kept {st['predictor_kept']}, "
          f"bitwise cold {same}; vs cold oracle T {eT:.2e} Y {eY:.2e}")
    assert np.all(st["per_state_status"] == 0)
    assert st["predictor_fallback"] >= 0.9 * len(rows)
    assert same >= st["predictor_fallback"]
    assert eT <= 1e-5 and eY <= 1e-5


def test_m150_block_options_and_step_limit(torch_dev, g150, o150):
    """The block kernel's Newton and step-size options (kmax 4, kappa 0.01,
    first step 1e-9 s) against the oracle with the same options, and the
    step-attempt limit: with nmax = 3 every state stops with STEP_LIMIT and
    keeps its last accepted solution, as the oracle does."""
    import oracle
    torch, _ = torch_dev
    banner("M150 block options kmax=4 kappa=0.01 h0=1e-9, nmax=3")
    rows = configs.states_for(configs.WORKLOADS["cfg4"], 40)
    g150.set_option("variant", "block")
    for k, v in (("kmax", "4"), ("kappa", "0.01"), ("h0", "1e-9")):
        g150.set_option(k, v)
    got = g150.integrate(_dev(torch_dev, rows), 1e-6).cpu().numpy().T
    st = g150.stats(per_state=True)
    for k, v in (("kmax", "7"), ("kappa", "0"), ("h0", "0")):
        g150.set_option(k, v)
    ref, res = o150.integrate(rows, 1e-6, opts=oracle.default_opts(kmax=4, kappa=0.01, h0=1e-9))
    eT, eY = integration_errors(got, ref, K)
    same = np.mean(st["per_state_steps"] == res["nstep"])
    print(f"M150 block options: T {eT:.2e} Y {eY:.2e}, identical step counts {same:.3f}")
    assert np.all(st["per_state_status"] == 0) and np.all(res["status"] == 0)
    assert eT <= 1e-5 and eY <= 1e-5 and same >= 0.95
    g150.set_option("nmax", "3")
    got = g150.integrate(_dev(torch_dev, rows), 1e-4).cpu().numpy().T
    st = g150.stats(per_state=True)
    g150.set_option("nmax", "100000")
    g150.set_option("variant", "auto")
    ref, res = o150.integrate(rows, 1e-4, opts=oracle.default_opts(nmax=3))
    print(f"M150 block nmax=3: status {np.bincount(st['per_state_status'])}, oracle {np.bincount(res['status'])}")
    assert np.all(st["per_state_status"] == 1) and np.all(res["status"] == 1)
    assert np.array_equal(st["per_state_steps"], res["nstep"])
    eT, eY = integration_errors(got, ref, K)
    assert eT <= 1e-5 and eY <= 1e-5
