"""fftg_apply_GK_noalloc (no plan, no device allocation, static scratch)
against fftg_apply_GK on a plan of the same grid, through the C ABI: two
calls in a row, the second on a smaller grid, in the IDENTITY and ELASTIC
forms; and the size and extent limits of the static scratch."""
import numpy as np
import pytest

import synth
from tests.gpu_util import rel_err, t2m, to_dev, to_host

pytestmark = pytest.mark.gpu

MATS = [(0.833, 0.386, 0.003, 0.004, 1.0), (2.0, 1.3, 0.006, 0.008, 1.0)]


def _plan_product(shape, p, mode, phase):
    from paper_1601_05970_amd import fftg
    opt = fftg.fftg_options_default()
    pl = fftg.Plan(phase, MATS, opt)
    out = pl.field()
    pl.apply_GK(to_dev(t2m(p)), out, mode)
    return to_host(out)


@pytest.mark.parametrize("mode_name", ["IDENTITY", "ELASTIC"])
@pytest.mark.parametrize("big,small", [((31, 25, 27), (15, 9, 21)), ((63, 63, 63), (5, 7, 3))])
def test_noalloc_equals_plan_product_two_calls(big, small, mode_name):
    import torch
    from paper_1601_05970_amd import fftg
    mode = getattr(fftg, "FFTG_TANGENT_" + mode_name)
    print("noalloc", mode_name, big, small, flush=True)
    cases = []
    for i, shape in enumerate((big, small)):
        p = synth.random_sym_tensor_field(shape, 40 + i)
        ph = synth.bernoulli(shape, 0.4, 50 + i)
        cases.append((shape, p, ph))
    outs = []
    for shape, p, ph in cases:   # two calls in a row, the second smaller
        d_in = to_dev(t2m(p))
        d_out = torch.full((6,) + shape, float("nan"), dtype=torch.float64, device="cuda")
        d_ph = torch.from_numpy(ph).cuda() if mode_name == "ELASTIC" else None
        fftg.fftg_apply_GK_noalloc(d_in, d_out, mode, d_ph, MATS if d_ph is not None else None)
        outs.append((d_in, d_out, d_ph))
    torch.cuda.synchronize()
    for (shape, p, ph), (_, d_out, _) in zip(cases, outs):
        ref = _plan_product(shape, p, mode, ph)
        assert rel_err(to_host(d_out), ref) < 1e-12, shape


def test_noalloc_limits():
    import torch
    from paper_1601_05970_amd import fftg
    print("noalloc limits", flush=True)
    for shape, status in (((75, 75, 75), fftg.FFTG_E_INVALID),       # half spectrum above 16 MiB - 64 KiB
                          ((127, 3, 5), fftg.FFTG_E_UNSUPPORTED),    # Rader extent
                          ((4, 5, 5), fftg.FFTG_E_INVALID)):         # even extent
        d_in = torch.zeros((6,) + shape, dtype=torch.float64, device="cuda")
        d_out = torch.zeros_like(d_in)
        with pytest.raises(fftg.FFTGError) as e:
            fftg.fftg_apply_GK_noalloc(d_in, d_out, fftg.FFTG_TANGENT_IDENTITY)
        assert e.value.status == status, shape
    d_in = torch.zeros((6, 5, 5, 5), dtype=torch.float64, device="cuda")
    with pytest.raises(fftg.FFTGError) as e:
        fftg.fftg_apply_GK_noalloc(d_in, torch.zeros_like(d_in), fftg.FFTG_TANGENT_CURRENT)
    assert e.value.status == fftg.FFTG_E_INVALID
