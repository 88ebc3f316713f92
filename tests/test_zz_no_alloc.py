"""The integrator's allocation-free entry point (ak_integrate_euler_noalloc,
scratch in a device array inside the library) against ak_integrate_euler,
through the C ABI: two calls in a row, the second with a smaller input;
identical results (the same kernels, whose accumulation order is fixed);
inputs beyond the scratch size are refused."""

import ctypes as C

import numpy as np
import pytest

from paper_2008_08483_amd import synth

pytestmark = pytest.mark.gpu

MILD = dict(ln_A_range=(8.0, 16.0), Ea_range=(20000.0, 60000.0))


def _fn(lib):
    f = lib.ak_integrate_euler_noalloc
    f.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                  C.c_int64, C.c_double, C.c_int, C.c_void_p]
    f.restype = C.c_int
    return f


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_matches_allocating_integrator(prec):
    import torch
    from paper_2008_08483_amd import annkin
    lib = annkin.lib()
    noalloc = _fn(lib)
    dt_t = torch.float64 if prec == "fp64" else torch.float32
    code = annkin.AK_FP64 if prec == "fp64" else annkin.AK_FP32
    src = synth.make_mechanism(53, 325, **MILD)
    m = annkin.Mechanism(src)
    assert m.compiled(dt_t)
    stream = torch.cuda.current_stream()
    for n, seed in ((5000, 31), (1234, 32)):        # second call smaller
        T, P, Y = synth.make_states(src, n, seed, (1000.0, 2500.0), (1.0, 20.0), 0.5)
        ref = [torch.tensor(a, dtype=dt_t, device="cuda") for a in (T, P, Y)]
        got = [r.clone() for r in ref]
        annkin.integrate_euler(m, ref[0], ref[1], ref[2], 5e-16, 20)
        rc = noalloc(m.handle, code, got[0].data_ptr(), got[1].data_ptr(), got[2].data_ptr(),
                     got[2].stride(0), n, 5e-16, 20, C.c_void_p(stream.cuda_stream))
        assert rc == 0, lib.ak_last_error()
        torch.cuda.synchronize()
        assert torch.equal(got[0], ref[0]) and torch.equal(got[2], ref[2])
        assert not torch.equal(got[0], torch.tensor(T, dtype=dt_t, device="cuda"))
    # more cells than the 64 MiB scratch holds: refused before any launch
    big = (64 << 20) // (53 * (8 if prec == "fp64" else 4)) + 1
    Tb = torch.ones(big, dtype=dt_t, device="cuda")
    Yb = torch.ones((53, big), dtype=dt_t, device="cuda")
    rc = noalloc(m.handle, code, Tb.data_ptr(), Tb.data_ptr(), Yb.data_ptr(), big, big, 1e-14,
                 1, C.c_void_p(stream.cuda_stream))
    assert rc == -4
    torch.cuda.synchronize()
    assert torch.all(Tb == 1)
    m.close()
