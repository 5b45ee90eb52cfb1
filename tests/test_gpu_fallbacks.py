"""GPU tests of paths the plain parity runs do not reach: the FP32 variants'
fallbacks forced from the host (the mixed variant's hand-back to the FP64
pass, also in place; the block variant's switch to FP64-accurate solves),
block-kernel refills (more states than blocks), the divergence statistics of
Eq. (3) recomputed from the per-state step counts, and the kernel-level
factorisation entry (rk_dbg_lu_solve) against LAPACK (FP64 factors) and the
backward-error bound of Gaussian elimination (FP32 factors)."""
import numpy as np
import pytest

from paper_1607_03884_amd import configs, gen
from tests.parity import banner, integration_errors

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch, torch.device("cuda:0")


def _dev(torch_dev, rows):
    torch, dev = torch_dev
    return torch.from_numpy(gen.to_soa(rows)).to(dev)


def _mech(name):
    from paper_1607_03884_amd import Mechanism
    return Mechanism(configs.mech_path(name))


CASES = {"M13": ("cfg0", 200), "M53": ("cfg2", 48)}


@pytest.mark.parametrize("name", ["M13", "M53"])
def test_mixed_forced_fallback_in_place(torch_dev, request, name):
    """Every state handed from the FP32 pass to the FP64 pass at its first
    accepted step, with y_out = y_in: the FP64 pass restarts from the
    untouched input, so the result is the FP64 variant's, bit for bit."""
    torch, _ = torch_dev
    om = request.getfixturevalue("m13" if name == "M13" else "m53")
    wl, n = CASES[name]
    rows = configs.states_for(configs.WORKLOADS[wl], n)
    K = configs.MECHS[name].n_species
    g = _mech(name)
    for dt in (1e-6, 1e-4):
        banner(f"{name} mixed forced fallback in place dt={dt}")
        g.set_option("variant", "wave")
        plain = g.integrate(_dev(torch_dev, rows), dt).cpu().numpy()
        g.set_option("variant", "mixed")
        g.set_option("force_fallback", "1")
        y = _dev(torch_dev, rows)
        g.integrate(y, dt, y_out=y)
        torch.cuda.synchronize()
        st = g.stats(per_state=True)
        got = y.cpu().numpy()
        assert st["fp32_fallback"] == n
        assert np.all(st["per_state_status"] == 0)
        assert np.array_equal(got, plain)
        ref, res = om.integrate(rows, dt)
        eT, eY = integration_errors(got.T, ref, K)
        assert eT <= TOL and eY <= TOL
        # the unforced mixed variant in place equals its out-of-place result
        g.set_option("force_fallback", "0")
        a = g.integrate(_dev(torch_dev, rows), dt).cpu().numpy()
        y = _dev(torch_dev, rows)
        g.integrate(y, dt, y_out=y)
        torch.cuda.synchronize()
        assert np.array_equal(a, y.cpu().numpy())
    g.close()


@pytest.fixture(scope="module")
def o150(oracle_mod):
    return oracle_mod.Mech(configs.mech_path("M150"))


@pytest.mark.parametrize("mode", ["refill", "forced", "fp64_accurate"])
def test_block_refill_and_fallbacks(torch_dev, o150, mode):
    """M150 on a tenth of the persistent grid (25 blocks), so every block
    integrates several states in turn and reuses its LDS, Jacobian slab and
    counters; with the FP64-accurate solves forced after the first accepted
    step, or from the first step.  Every state against the oracle."""
    torch, _ = torch_dev
    K = 150
    n = 160 if mode == "refill" else 67
    rows = configs.states_for(configs.WORKLOADS["cfg4"], n)
    g = _mech("M150")
    g.set_option("variant", "block")
    g.set_option("grid_pct", "10")
    if mode == "forced":
        g.set_option("force_fallback", "1")
    if mode == "fp64_accurate":
        g.set_option("block_solves", "fp64_accurate")
    for dt in ((1e-6, 1e-4) if mode == "refill" else (1e-4,)):
        banner(f"M150 block {mode} {n} states dt={dt}")
        out = g.integrate(_dev(torch_dev, rows), dt, configs.ATOL, configs.RTOL)
        torch.cuda.synchronize()
        st = g.stats(per_state=True)
        got = out.cpu().numpy().T
        assert st["grid_used"] < n
        ref, res = o150.integrate(rows, dt)
        assert np.all(res["status"] == 0) and np.all(st["per_state_status"] == 0)
        eT, eY = integration_errors(got, ref, K)
        same = np.mean(st["per_state_steps"] == res["nstep"])
        print(f"M150 block {mode}: grid {st['grid_used']}, kernel {st['kernel_ms']:.1f} ms, "
              f"max rel err T {eT:.2e} Y {eY:.2e}, identical step counts {same:.3f}, "
              f"fp32_fallback {st['fp32_fallback']}")
        assert eT <= TOL and eY <= TOL
        if mode == "forced":
            # every state that took a step after its first accepted one switched
            assert st["fp32_fallback"] == int(np.sum(st["per_state_steps"] > 1)) > 0
        elif mode == "fp64_accurate":
            assert st["fp32_fallback"] == n
    g.close()


def test_divergence_statistics_match_eq3(torch_dev):
    """stats_get's D histograms and means (Eq. 3 over groups of 64 and 32
    consecutive states) against a recomputation from the per-state step
    counts; the queue-order measure equals the input-order one without bins
    and is lower with cost bins (the bins group states of equal cost)."""
    torch, _ = torch_dev
    banner("D statistics M13 cfg1 subset")
    rows = configs.states_for(configs.WORKLOADS["cfg1"], 8192 + 37)
    g = _mech("M13")

    def eq3(steps, w):
        hist = np.zeros(20, dtype=np.int64)
        Ds = []
        for g0 in range(0, len(steps), w):
            d = steps[g0:g0 + w].astype(np.float64)
            D = 1.0 - d.sum() / (len(d) * d.max())
            hist[min(19, max(0, int(D / 0.05)))] += 1
            Ds.append(D)
        return hist, float(np.mean(Ds))

    for bins in (0, 16):
        g.set_option("binning", str(bins))
        g.integrate(_dev(torch_dev, rows), 1e-4)
        torch.cuda.synchronize()
        st = g.stats(per_state=True)
        steps = st["per_state_steps"]
        for w, key in ((64, "64"), (32, "32")):
            h, mean = eq3(steps, w)
            assert list(h) == st[f"d_hist{key}"]
            assert abs(mean - st[f"d_mean{key}"]) <= 1e-12
        if bins == 0:
            assert st["d_hist64_queue"] == st["d_hist64"]
            assert st["d_mean64_queue"] == st["d_mean64"]
        else:
            assert sum(st["d_hist64_queue"]) == sum(st["d_hist64"])
            assert st["d_mean64_queue"] < st["d_mean64"]
        print(f"bins {bins}: D64 input order {st['d_mean64']:.3f}, queue order {st['d_mean64_queue']:.3f}")
    g.close()


def _equilibrated(E, sc):
    """The documented equilibration of the FP32 factors: columns by sc_c, rows
    by 1/sc_r and then by the power of two at or below the row's largest real
    or imaginary magnitude.  Returns E'' and the row factors d_r (E'' = D E S)."""
    Es = E * sc[None, :] / sc[:, None]
    m = np.maximum(np.abs(Es.real).max(axis=1), np.abs(np.imag(Es)).max(axis=1))
    p = 2.0 ** np.floor(np.log2(m))
    return Es / p[:, None], 1.0 / (sc * p)


@pytest.mark.parametrize("name", ["M13", "M53"])
def test_lu_solve_entry(torch_dev, name):
    """rk_dbg_lu_solve: FP64 factors against LAPACK's solve of E1 and E2
    (forward error within cond(E) u); FP32 factors (no refinement) within the
    normwise backward-error bound of partial-pivoting elimination, c N 2^-24,
    in the equilibrated coordinates they factor (c = 16)."""
    torch, dev = torch_dev
    banner(f"lu_solve entry {name}")
    g = _mech(name)
    N = g.N
    wl = "cfg1" if name == "M13" else "cfg2"
    rows = configs.states_for(configs.WORKLOADS[wl], 40)
    y = _dev(torch_dev, rows)
    J = g.dbg_jacobian(y)
    n = rows.shape[0]
    rng = np.random.default_rng(5)
    b = rng.standard_normal((3 * N, n))
    sc = 1e-10 + 1e-6 * np.abs(rows[:, :N].T)
    Jh = J.cpu().numpy().T.reshape(n, N, N)
    from oracle import radau_constants
    consts = radau_constants()
    gam, alp, bet = consts["gamma"], consts["alpha"], consts["beta"]
    worst64 = worst32 = 0.0
    for h in (1e-9, 1e-7, 1e-5):
        x64 = g.dbg_lu_solve(J, torch.from_numpy(b).to(dev), h, fp32=False).cpu().numpy()
        x32 = g.dbg_lu_solve(J, torch.from_numpy(b).to(dev), h, fp32=True,
                             sc=torch.from_numpy(np.ascontiguousarray(sc)).to(dev)).cpu().numpy()
        for i in range(n):
            E1 = gam / h * np.eye(N) - Jh[i]
            E2 = (alp + 1j * bet) / h * np.eye(N) - Jh[i]
            b1, b2 = b[:N, i], b[N:2 * N, i] + 1j * b[2 * N:, i]
            for E, bb, xg, x3 in ((E1, b1, x64[:N, i], x32[:N, i]),
                                  (E2, b2, x64[N:2 * N, i] + 1j * x64[2 * N:, i],
                                   x32[N:2 * N, i] + 1j * x32[2 * N:, i])):
                xr = np.linalg.solve(E, bb)
                cond = np.linalg.cond(E, np.inf)
                fe = np.abs(xg - xr).max() / np.abs(xr).max()
                assert fe <= 64 * N * cond * np.finfo(float).eps, (h, i, fe, cond)
                worst64 = max(worst64, fe / cond)
                # FP32: backward error in the equilibrated coordinates
                Ee, d = _equilibrated(E, sc[:, i])
                be = bb * d
                xe = x3 / sc[:, i]
                r = be - Ee @ xe
                eta = np.abs(r).max() / (np.abs(Ee).sum(axis=1).max() * np.abs(xe).max() + np.abs(be).max())
                assert eta <= 16 * N * 2.0 ** -24, (h, i, eta)
                worst32 = max(worst32, eta)
    print(f"{name}: FP64 forward error / cond <= {worst64:.2e}; FP32 backward error <= {worst32:.2e} "
          f"(bound {8 * N * 2.0 ** -24:.2e})")
    g.close()
