"""The benchmarked learned form against the cold-started oracle, at full size.

The learned form (FP32 iteration-matrix factors with FP64 residuals, a
persistent queue ordered by bins of the network's predicted step counts) does
not warm-start any state: the network only orders the queue.  Every state's
result is therefore bitwise that of the same variant without the predictor,
and it is held to the acceptance bar against the plain FP64 oracle started
cold: max relative error <= 1e-5 on T and on every Y_i whose oracle value
exceeds 1e-8 (atol 1e-10, rtol 1e-6).  Checked on a sample of every full
workload: the 1 % costliest states (by step count) and a seeded random draw."""
import numpy as np
import pytest

from paper_1607_03884_amd import configs, gen, predictor
from tests.parity import banner, integration_errors

pytestmark = pytest.mark.gpu

TOL = 1e-5
DTS = [1e-6, 1e-4]


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch, torch.device("cuda:0")


def _run(torch_dev, g, y, dt):
    torch, _ = torch_dev
    out = torch.full_like(y, float("nan"))
    g.integrate(y, dt, configs.ATOL, configs.RTOL, y_out=out)
    torch.cuda.synchronize()
    return out.cpu().numpy().T, g.stats(per_state=True)


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("wl,mname,nrand", [("cfg1", "M13", 1024), ("cfg3", "M53", 512)])
def test_learned_form_matches_cold_oracle(torch_dev, request, wl, mname, nrand, dt):
    torch, dev = torch_dev
    from paper_1607_03884_amd import Mechanism
    om = request.getfixturevalue("m13" if mname == "M13" else "m53")
    rows = configs.states_for(configs.WORKLOADS[wl])
    K = configs.MECHS[mname].n_species
    n = len(rows)
    banner(f"learned form {wl} ({n} states) dt={dt} vs cold oracle")
    y = torch.from_numpy(gen.to_soa(rows)).to(dev)
    g = Mechanism(configs.mech_path(mname))
    g.set_option("variant", "mixed")
    base, sb = _run(torch_dev, g, y, dt)
    g.set_option("predictor", predictor.path_for(mname, dt))
    g.set_option("predictor_use", "bins")
    g.set_option("binning", "16")
    got, st = _run(torch_dev, g, y, dt)
    g.close()
    print(f"{wl} dt={dt}: mixed input order {sb['kernel_ms']:.1f} ms, learned form {st['kernel_ms']:.1f} ms; "
          f"D64 queue order {st['d_mean64_queue']:.3f} vs input order {st['d_mean64']:.3f}; "
          f"fp32 fallback {st['fp32_fallback']}")
    assert np.all(st["per_state_status"] == 0)
    assert st["nbins_used"] == 16
    assert st["predictor_kept"] == 0 and st["predictor_fallback"] == 0
    # the network orders the queue and nothing else
    assert np.array_equal(got, base)
    assert np.array_equal(st["per_state_steps"], sb["per_state_steps"])
    steps = st["per_state_steps"]
    top = np.argsort(steps, kind="stable")[-max(1, n // 100):]
    rng = np.random.default_rng(2024)
    pick = np.unique(np.concatenate([top, rng.choice(n, nrand, replace=False)]))
    ref, res = om.integrate(rows[pick], dt)
    assert np.all(res["status"] == 0)
    eT, eY = integration_errors(got[pick], ref, K)
    same = np.mean(steps[pick] == res["nstep"])
    print(f"  {len(pick)} states (1 % costliest + {nrand} random): max rel err T {eT:.2e} Y {eY:.2e}, "
          f"identical step counts {same:.4f}")
    assert eT <= TOL and eY <= TOL
