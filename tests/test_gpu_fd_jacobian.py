"""GPU Radau IIA with the first-order forward-difference Jacobian (the
alternative Sec. 3.4 compares with the analytical Jacobian), lane-per-state
and wavefront-cooperative kernels, against the oracle with the same
Jacobian rule; the extra source-term evaluations are counted."""
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


CASES = [("M13", "cfg1", 512, "lane"), ("M13", "cfg1", 512, "wave"), ("M53", "cfg2", 64, "wave")]


@pytest.mark.parametrize("dt", [1e-6, 1e-4])
@pytest.mark.parametrize("name,wl,n,variant", CASES)
def test_fd_jacobian_parity(torch_dev, request, name, wl, n, variant, dt):
    torch, dev = torch_dev
    from oracle import default_opts
    from paper_1607_03884_amd import Mechanism
    om = request.getfixturevalue("m13" if name == "M13" else "m53")
    K = configs.MECHS[name].n_species
    banner(f"fd jacobian {name} {variant} n={n} dt={dt}")
    rows = configs.states_for(configs.WORKLOADS[wl], n)
    g = Mechanism(configs.mech_path(name))
    g.set_option("variant", variant)
    g.set_option("jacobian", "fd")
    y = torch.from_numpy(gen.to_soa(rows)).to(dev)
    out = g.integrate(y, dt, configs.ATOL, configs.RTOL)
    torch.cuda.synchronize()
    st = g.stats(per_state=True)
    got = out.cpu().numpy().T
    g.set_option("jacobian", "analytical")
    g.integrate(y, dt, configs.ATOL, configs.RTOL)
    torch.cuda.synchronize()
    sa = g.stats()
    g.close()
    ref, res = om.integrate(rows, dt, opts=default_opts(fd_jac=1))
    assert np.all(res["status"] == 0) and np.all(st["per_state_status"] == 0)
    eT, eY = integration_errors(got, ref, K)
    same = np.mean(st["per_state_steps"] == res["nstep"])
    print(f"{name} {variant} dt={dt}: FD vs oracle FD: T {eT:.2e} Y {eY:.2e}, identical step counts {same:.4f}; "
          f"f-evals FD {st['f_evals']} vs analytical {sa['f_evals']}, Jacobians {st['jac_evals']} / {sa['jac_evals']}")
    assert eT <= TOL and eY <= TOL
    # a forward-difference Jacobian costs N = K + 1 source-term evaluations
    assert st["f_evals"] >= sa["f_evals"] - 3 * st["newton_iters"] + (K + 1) * st["jac_evals"] * 0.5


def test_fd_jacobian_refused_for_fp32_variants(torch_dev):
    torch, dev = torch_dev
    banner("fd jacobian refused for mixed")
    from paper_1607_03884_amd import Mechanism
    from paper_1607_03884_amd._lib import RkError
    g = Mechanism(configs.mech_path("M13"))
    g.set_option("variant", "mixed")
    g.set_option("jacobian", "fd")
    rows = configs.states_for(configs.WORKLOADS["cfg0"], 8)
    with pytest.raises(RkError):
        g.integrate(torch.from_numpy(gen.to_soa(rows)).to(dev), 1e-6)
    with pytest.raises(RkError):
        g.set_option("jacobian", "numerical")
    g.close()


@pytest.mark.parametrize("dt", [1e-6, 1e-4])
@pytest.mark.parametrize("name,wl,n", [("M13", "cfg1", 2048), ("M53", "cfg2", 256)])
def test_rodas3_parity(torch_dev, request, name, wl, n, dt):
    """The Rosenbrock method (Rodas3, the direction Sec. 4 recommends) on the
    wavefront kernels against the oracle's Rodas3: same step sequence, results
    to the acceptance bar; linear invariants to rounding; schedule invariance."""
    torch, dev = torch_dev
    from paper_1607_03884_amd import Mechanism
    om = request.getfixturevalue("m13" if name == "M13" else "m53")
    K = configs.MECHS[name].n_species
    banner(f"rodas3 {name} n={n} dt={dt}")
    rows = configs.states_for(configs.WORKLOADS[wl], n)
    g = Mechanism(configs.mech_path(name))
    g.set_option("method", "rodas3")
    y = torch.from_numpy(gen.to_soa(rows)).to(dev)
    out = g.integrate(y, dt, configs.ATOL, configs.RTOL)
    torch.cuda.synchronize()
    st = g.stats(per_state=True)
    got = out.cpu().numpy().T
    g.set_option("binning", "8")
    g.set_option("tile", "2")
    binned = g.integrate(y, dt, configs.ATOL, configs.RTOL).cpu().numpy().T
    g.close()
    ref, res = om.integrate_rodas3(rows, dt)
    assert np.all(res["status"] == 0) and np.all(st["per_state_status"] == 0)
    assert np.array_equal(binned, got)
    eT, eY = integration_errors(got, ref, K)
    same = np.mean(st["per_state_steps"] == res["nstep"])
    print(f"rodas3 {name} dt={dt}: vs oracle T {eT:.2e} Y {eY:.2e}, identical step counts {same:.4f}, "
          f"steps/state {st['steps'] / n:.1f}, kernel {st['kernel_ms']:.1f} ms")
    assert eT <= TOL and eY <= TOL
    assert same >= 0.98
    assert st["newton_iters"] == 0
    assert np.abs(got[:, 1:K + 1].sum(1) - rows[:, 1:K + 1].sum(1)).max() <= 1e-12
