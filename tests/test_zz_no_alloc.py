"""md_forces_noalloc (per-call scratch in the library's static device array, no device
allocation) against md_forces through the C ABI: identical results bit for bit, on two calls in a
row with the second on a smaller system, for the single-site full-shell kernel and the
multi-site half-shell kernel in both precisions; a configuration beyond the array's size is
rejected with nothing written."""
import numpy as np
import pytest
import torch

from tests._gpu import dev
from paper_1408_4599_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def md():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1408_4599_amd import md as _md
    _md.lib()
    return _md


def _alloc(N, fill):
    t = lambda shape, dtype=torch.float64: torch.full(shape, fill, dtype=dtype, device="cuda")
    return {"force": t((N, 3)), "torque": t((N, 3)), "u_mol": t((N,)), "w_mol": t((N,)),
            "nnb": torch.full((N,), -5, dtype=torch.int32, device="cuda"), "uw": t((5,)),
            "npairs": torch.full((1,), -5, dtype=torch.int64, device="cuda")}


def _both(md, cfg, prec):
    m = md.Model(cfg["model"])
    cells = md.Cells()
    ncomp = len(cfg["model"]["components"])
    md.build_cells(m, cells, dev(cfg["pos"]), dev(cfg["quat"]), dev(cfg["comp"], torch.int32) if ncomp > 1 else None,
                   cfg["box"])
    N = cfg["pos"].shape[0]
    a, b = _alloc(N, 3.0), _alloc(N, -7.0)
    md.forces_into(m, cells, prec, a)
    md.forces_into_noalloc(m, cells, prec, b)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in a.items()}, {k: v.cpu().numpy() for k, v in b.items()}


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("first,second", [("c1_ljts_4000", "lj_gas_2500"), ("c4_small", "four_site_900")])
def test_noalloc_equals_forces_on_two_calls(md, first, second, prec):
    small = {"lj_gas_2500": lambda: W.random_gas(2500, [15.0, 16.0, 17.0], W.lj_model(2.5), seed=21, dmin=0.9),
             "four_site_900": lambda: W.random_gas(900, [13.0, 13.5, 14.0], W.four_site_model(), seed=23, dmin=1.0)}
    for name in (first, second):
        cfg = small[name]() if name in small else W.make(name)
        print(f"{name} {prec}: N={cfg['pos'].shape[0]}", flush=True)
        a, b = _both(md, cfg, prec)
        assert a["npairs"][0] > 0
        for k in a:
            np.testing.assert_array_equal(b[k], a[k], err_msg=f"{name} {prec} {k}")


def test_noalloc_rejects_beyond_the_array(md):
    """FP64 multi-site with per-molecule outputs needs 1080 B per molecule of partner rows: 20 000
    molecules exceed the 16 MiB array.  The call fails with MD_EINVAL and writes nothing."""
    cfg = W.random_gas(20000, [46.0, 46.0, 46.0], W.four_site_model(), seed=25, dmin=0.9)
    m = md.Model(cfg["model"])
    cells = md.Cells()
    md.build_cells(m, cells, dev(cfg["pos"]), dev(cfg["quat"]), None, cfg["box"])
    out = _alloc(20000, 3.0)
    with pytest.raises(md.MDError) as e:
        md.forces_into_noalloc(m, cells, "fp64", out)
    assert e.value.code == md.MD_EINVAL and "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert bool((out["force"] == 3.0).all())
    # without per-molecule outputs FP32 fits (360 B per molecule)
    small = {k: out[k] for k in ("force", "torque", "uw", "npairs")}
    md.forces_into_noalloc(m, cells, "fp32", small)
    ref = md.forces(m, cells, "fp32", per_molecule=False)
    torch.cuda.synchronize()
    for k in ("force", "torque", "uw", "npairs"):
        assert torch.equal(small[k], ref[k]), k
