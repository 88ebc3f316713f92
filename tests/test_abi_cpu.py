"""Host-only checks of the C ABI: the library loads, exports every function
include/annkin.h declares, and rejects bad arguments before touching a GPU."""

import ctypes as C
import os
import re

import numpy as np

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "annkin.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ak_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2008_08483_amd import annkin
    return annkin.lib()


def test_header_declares_entry_points():
    names = declared_functions()
    for required in ("ak_load_mechanism", "ak_eval_source", "ak_free_mechanism",
                     "ak_last_error", "ak_error_count"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_argument_errors_without_gpu(lib):
    from paper_2008_08483_amd import annkin
    out = C.c_void_p()
    assert lib.ak_load_mechanism(None, 0, C.byref(out)) == -1
    assert b"null" in lib.ak_last_error()
    d = annkin.MechanismDesc()
    d.n_species = 0
    assert lib.ak_load_mechanism(C.byref(d), 0, C.byref(out)) == -1
    d.n_species, d.n_reactions = 257, 1          # species indices are bytes
    assert lib.ak_load_mechanism(C.byref(d), 0, C.byref(out)) == -7
    assert b"257 species" in lib.ak_last_error()
    assert lib.ak_eval_source(None, 0, None, None, None, 0, 0, None, 0, None) == -1
    assert lib.ak_free_mechanism(None) == 0
    assert lib.ak_eval_production(None, None, 0, 0, None, 0, None) == -1
    assert lib.ak_mechanism_n_species(None) == -1
    assert lib.ak_version().startswith(b"annkin")


def test_server_submit_rejects_mismatched_buffers():
    """Server.submit checks dtypes, shapes and contiguity of every host buffer
    before anything reaches the library (no GPU needed)."""
    import numpy as np
    import pytest
    from paper_2008_08483_amd import annkin

    class _M:
        n_species = 3
        handle = None

    srv = object.__new__(annkin.Server)   # never created: submit must raise first
    n = 8
    Y = np.zeros((3, n), np.float64)
    T = np.ones(n)
    P = np.ones(n)
    out = np.zeros((3, n))
    bad = [
        (T.astype(np.float32), P, Y, out, TypeError),          # T dtype
        (T, P.astype(np.float32), Y, out, TypeError),          # P dtype
        (T, P, Y, out.astype(np.float32), TypeError),          # out dtype
        (T[:4], P, Y, out, ValueError),                        # T length
        (np.ones(2 * n)[::2], P, Y, out, ValueError),          # T not contiguous
        (T, P, Y, np.zeros((3, 2 * n))[:, ::2], ValueError),   # out cell stride
        (T, P, np.zeros((2, n)), out, ValueError),             # Y species count
        (T.astype(np.int32), P.astype(np.int32), Y.astype(np.int32), out, TypeError),
    ]
    for t, p, y, o, exc in bad:
        with pytest.raises(exc):
            srv.submit(_M(), t, p, y, o)


def test_pressure_dependent_descriptor_checks():
    """Third-body / falloff fields are validated at load (host only: the
    source generator runs the same checks without a GPU)."""
    import numpy as np
    from paper_2008_08483_amd import annkin, synth

    base = synth.with_pressure_dependence(synth.make_mechanism(9, 21), frac=0.5)
    text = annkin.jit_source(base, "fp64")
    assert "Ctot" in text and "lM" in text and "exp2(" in text   # [M] and the falloff epilogue
    text32 = annkin.jit_source(base, "fp32")
    assert "__builtin_amdgcn_exp2f" in text32

    def variant(**kw):
        import copy
        m = copy.copy(base)
        for k, v in kw.items():
            setattr(m, k, v)
        return m

    bad_type = base.rtype.copy()
    bad_type[0] = 4
    neg_eff = base.eff.copy()
    neg_eff[np.nonzero(base.rtype)[0][0], 0] = -1.0
    j_troe = int(np.nonzero(base.rtype == 3)[0][0])
    bad_troe = base.troe.copy()
    bad_troe[j_troe, 1] = 0.0
    for m in (variant(rtype=bad_type), variant(eff=neg_eff), variant(troe=bad_troe),
              variant(low_ln_A=None, low_beta=None, low_Ea=None), variant(troe=None)):
        with pytest.raises(annkin.AnnkinError) as e:
            annkin.jit_source(m, "fp32")
        assert e.value.code == -1, annkin.lib().ak_last_error()


def test_compiled_jacobian_generation_without_gpu():
    """The Jacobian generator runs on the host: both layouts, one kernel, the
    tables' sizes (32 doubles per species, 4 per reaction), and the refusal
    of pressure-dependent mechanisms."""
    from paper_2008_08483_amd import annkin, synth

    src = synth.make_mechanism(9, 21)
    for prec in ("fp32", "fp64"):
        a = annkin.jit_jacobian_source(src, prec)
        b = annkin.jit_jacobian_source(src, prec, interleaved=True)
        assert 'extern "C" __global__' in a and "void ak_jac(" in a
        assert "cell-major J" in a and "interleaved J" in b
        assert a.count("__syncthreads()") == b.count("__syncthreads()")
    sp, rx = annkin.jit_jacobian_tables(src)
    assert sp.shape == (32 * 9,) and rx.shape == (4 * 21,)
    # NASA-7 sets copied as given: low range of species 0
    assert np.allclose(sp[16:23], src.nasa_low[0])
    pd = synth.with_pressure_dependence(src, frac=0.5)
    with pytest.raises(annkin.AnnkinError) as e:
        annkin.jit_jacobian_source(pd, "fp64")
    assert e.value.code == -7


def test_kcnet_descriptor_refusals_without_gpu():
    # ak_load_kcnet checks the descriptor before it touches a device
    import ctypes as C

    from paper_2008_08483_amd import annkin, kcnet
    h = annkin.lib()
    net = kcnet.random_weights(2, 8, 5, seed=1)
    w = np.concatenate([a.reshape(-1) for a in net.weights])
    b = np.concatenate(net.biases)
    ym, ys = np.ascontiguousarray(net.y_mean), np.ascontiguousarray(net.y_std)

    def load(nl=2, nh=8, nr=5, ww=w, xstd=net.x_std):
        d = annkin.KcNetDesc(nl, nh, nr, 0, ww.ctypes.data, b.ctypes.data, net.x_mean, xstd,
                             ym.ctypes.data, ys.ctypes.data)
        out = C.c_void_p()
        return h.ak_load_kcnet(C.byref(d), 0, C.byref(out))

    assert load(nh=65) == -1
    assert load(nl=0) == -1
    assert load(nl=17) == -1
    assert load(nr=0) == -1
    assert load(xstd=0.0) == -1
    bad = w.copy()
    bad[3] = np.nan
    assert load(ww=bad) == -1
    assert "non-finite weight" in h.ak_last_error().decode()
