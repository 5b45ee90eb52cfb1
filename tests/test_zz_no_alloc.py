"""radau_integrate_noalloc (the entry point for callers that cannot allocate)
against radau_integrate: same kernels, so the same bits, on two calls in a
row with the second smaller; the oracle's acceptance bar on the first; the
size limit and the refused variants; and no change of the device's free
memory across a call on a fresh handle."""
import numpy as np
import pytest

from paper_1607_03884_amd import configs, gen
from tests.parity import banner, integration_errors

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch, torch.device("cuda:0")


def _dev(torch_dev, rows):
    torch, dev = torch_dev
    return torch.from_numpy(gen.to_soa(rows)).to(dev)


@pytest.mark.parametrize("name,wl,sizes,variant", [("M13", "cfg1", (3000, 777), "wave"),
                                                   ("M13", "cfg1", (2048, 130), "mixed"),
                                                   ("M53", "cfg2", (96, 40), "mixed")])
def test_noalloc_matches_radau_integrate(torch_dev, request, name, wl, sizes, variant):
    torch, _ = torch_dev
    from paper_1607_03884_amd import Mechanism
    om = request.getfixturevalue("m13" if name == "M13" else "m53")
    K = configs.MECHS[name].n_species
    rows = configs.states_for(configs.WORKLOADS[wl], max(sizes))
    g = Mechanism(configs.mech_path(name))
    g.set_option("variant", variant)
    for call, n in enumerate(sizes):
        for dt in (1e-6, 1e-4):
            banner(f"noalloc {name} {variant} call {call} n={n} dt={dt}")
            y = _dev(torch_dev, rows[:n])
            ref = g.integrate(y, dt)
            torch.cuda.synchronize()
            sr = g.stats(per_state=True)
            out = torch.full_like(y, float("nan"))
            g.integrate_noalloc(y, dt, y_out=out)
            torch.cuda.synchronize()
            st = g.stats(per_state=True)
            assert torch.equal(out, ref)
            assert np.array_equal(st["per_state_steps"], sr["per_state_steps"])
            assert np.array_equal(st["per_state_status"], sr["per_state_status"])
            assert st["n_states"] == n and st["nbins_used"] == 0
            if call == 0 and dt == 1e-6:
                sub = rows[:min(n, 256)]
                oref, res = om.integrate(sub, dt)
                eT, eY = integration_errors(out.cpu().numpy().T[:len(sub)], oref, K)
                assert eT <= 1e-5 and eY <= 1e-5
    g.close()


def test_noalloc_limits_and_refusals(torch_dev):
    torch, dev = torch_dev
    banner("noalloc limits")
    from paper_1607_03884_amd import Mechanism
    from paper_1607_03884_amd._lib import RkError
    g = Mechanism(configs.mech_path("M13"))
    big = torch.zeros((15, 262145), dtype=torch.float64, device=dev)
    with pytest.raises(RkError, match="262144"):
        g.integrate_noalloc(big, 1e-6, y_out=big)
    del big
    empty = torch.zeros((15, 0), dtype=torch.float64, device=dev)
    g.integrate_noalloc(empty, 1e-6, y_out=empty)
    assert g.stats()["n_states"] == 0
    rows = configs.states_for(configs.WORKLOADS["cfg0"], 8)
    for v in ("lane", "block"):
        g.set_option("variant", v)
        with pytest.raises(RkError):
            g.integrate_noalloc(_dev(torch_dev, rows), 1e-6)
    g.close()


def test_noalloc_leaves_free_memory_unchanged(torch_dev):
    """A call on a fresh handle (no workspace of its own yet) changes the
    device's free memory by nothing: the static array was placed when the
    library's code was loaded."""
    torch, dev = torch_dev
    banner("noalloc free memory")
    from paper_1607_03884_amd import Mechanism
    rows = configs.states_for(configs.WORKLOADS["cfg1"], 4096)
    y = _dev(torch_dev, rows)
    out = torch.empty_like(y)
    g0 = Mechanism(configs.mech_path("M13"))
    g0.integrate_noalloc(y, 1e-6, y_out=out)     # loads the code, places the array
    torch.cuda.synchronize()
    g = Mechanism(configs.mech_path("M13"))
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    g.integrate_noalloc(y, 1e-6, y_out=out)
    torch.cuda.synchronize()
    g.stats()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0
    g.close()
    g0.close()
