"""exo_cross_section_noalloc: the cross-section that allocates nothing, against
exo_cross_section (the same kernels on the context's workspace), through the
C ABI.  Two calls in a row, the second on a smaller input, each checked
element by element; then a call beyond the scratch's limit is refused."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def exo():
    import paper_2105_14782_amd as pkg
    pkg.load_library()
    from paper_2105_14782_amd import api
    return api


def _lines(rng, n, lo, hi):
    return synth.LineList(np.sort(rng.uniform(lo, hi, n)), 10 ** rng.uniform(-25, -19, n),
                          rng.exponential(2000, n), rng.uniform(0.01, 0.1, n), rng.uniform(0.5, 0.8, n),
                          18.0, 0, np.array([1.5]))


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_noalloc_matches_cross_section_twice(exo, prec):
    rng = np.random.default_rng(77)
    c = exo.Context(0)
    c.set_lines(0, _lines(rng, 3000, 4335.0, 4365.0))
    c.set_lines(1, _lines(rng, 137, 4342.0, 4351.0))      # the smaller second input
    nu = np.linspace(4340.0, 4360.0, 5003)
    c.set_grid(nu)
    dt = torch.float64 if prec == "fp64" else torch.float32
    for slot, T, P in [(0, 1500.0, 0.3), (1, 700.0, 2.0)]:
        ref = c.cross_section(slot, T, P, prec)
        out = torch.full((nu.size,), float("nan"), dtype=dt, device="cuda")
        c.cross_section_noalloc(slot, T, P, out, prec)
        torch.cuda.synchronize()
        r, o = ref.cpu().double().numpy(), out.cpu().double().numpy()
        err = float(np.max(np.abs(o - r) / np.abs(r)))
        print(f"  {prec} slot {slot}: max rel diff to exo_cross_section {err:.1e}", flush=True)
        assert err < (1e-4 if prec == "fp32" else 1e-5)
        assert torch.equal(out.cpu(), ref.cpu())          # the same kernels and launch shapes
    c.close()


def test_noalloc_refuses_beyond_its_scratch(exo):
    import paper_2105_14782_amd as pkg
    rng = np.random.default_rng(78)
    c = exo.Context(0)
    c.set_lines(0, _lines(rng, 2_500_000, 4000.0, 4700.0))   # 160 MB of FP32 records
    c.set_grid(np.linspace(4340.0, 4360.0, 1000))
    out = torch.zeros(1000, dtype=torch.float32, device="cuda")
    with pytest.raises(pkg.ExoError) as e:
        c.cross_section_noalloc(0, 1000.0, 1.0, out)
    assert e.value.code == pkg.EXO_ENOMEM
    assert "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert torch.count_nonzero(out).item() == 0              # nothing was launched
    c.close()
