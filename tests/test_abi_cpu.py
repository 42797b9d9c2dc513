"""CPU checks of the boundary: the built library loads and exports every
entry point include/fftg.h declares; host-only calls work without a GPU."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1601_05970_amd", "libfftg.so")


def declared():
    text = open(os.path.join(ROOT, "include", "fftg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fftg_[a-zA-Z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("libfftg.so not built")
    from paper_1601_05970_amd import fftg
    return fftg.lib()


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_the_header():
    from paper_1601_05970_amd import fftg
    assert sorted(fftg.EXPORTS) == declared()


def test_host_only_calls(lib):
    from paper_1601_05970_amd import fftg
    o = fftg.fftg_options_default()
    assert o.tol_newton == 1e-5 and o.tol_cg == 1e-8 and o.predictor == 0
    f64 = fftg.fftg_footprint_bytes(127, 127, 127, fftg.FFTG_FP64)
    f32 = fftg.fftg_footprint_bytes(127, 127, 127, fftg.FFTG_MIXED)
    assert 0 < f32 < f64 < 2 ** 31
    assert fftg.fftg_footprint_bytes(0, 1, 1, 0) == 0
    assert lib.fftg_last_error() is not None
    # sampled kernel timing: bad kernel ids and strides are rejected
    for kid, every in ((fftg.FFTG_KERNEL_ZFWD, 0), (-1, 1), (8, 1)):
        with pytest.raises(fftg.FFTGError):
            fftg.fftg_profiler_start_every(kid, every)


def test_struct_layouts_match_header():
    import ctypes as C
    from paper_1601_05970_amd import fftg
    assert C.sizeof(fftg.fftg_material) == 64
    assert C.sizeof(fftg.fftg_options) == 80
    assert C.sizeof(fftg.fftg_stats) == 4 + 4 * 64 + 4 + 8 * 64 + 8 * 6 + 4 + 4 + 8 + 8
