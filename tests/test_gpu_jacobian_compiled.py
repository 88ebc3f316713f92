"""The state Jacobian compiled for the mechanism (one 64-cell tile per
workgroup, every sum in a fixed order), through the C ABI: parity against the
oracle in both output layouts (cell-major and interleaved), bitwise equality
of the two layouts and of repeated calls, agreement with the table-driven
kernel, ragged tiles, strides, bad cells, and the paths it refuses.

Tolerances as in tests/test_gpu_deriv.py: each entry's error against the
oracle's gross scale of that entry, <= 1e-11 for FP64 (against the
extended-precision oracle), <= 1e-6 for FP32 output (double inside).
"""

import dataclasses
import os

import numpy as np
import pytest

import oracle
from paper_2008_08483_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.fixture(scope="module")
def ak():
    from paper_2008_08483_amd import annkin
    return annkin


_MECHS = {}


def _mech(ak, ns, nr, irreversible=0.0):
    key = (ns, nr, irreversible)
    if key not in _MECHS:
        src = synth.make_mechanism(ns, nr)
        if irreversible:
            rev = src.reversible.copy()
            rev[np.random.default_rng(31).random(nr) < irreversible] = 0
            src = dataclasses.replace(src, reversible=rev)
        _MECHS[key] = (src, ak.Mechanism(src))
    return _MECHS[key]


def _dev(torch, dt, *arrs):
    return [torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda") for a in arrs]


def _check(src, T, P, Y, J, tol):
    Jr, Ja = oracle.jacobian(src, T, P, Y, precision="ld", scales=True)
    err = np.abs(J.astype(np.longdouble) - Jr) / np.maximum(Ja, np.longdouble(1e-300))
    e = float(err.max())
    print("jacobian max err/scale", e, flush=True)
    assert np.all(np.isfinite(J))
    assert e <= tol


@pytest.mark.parametrize("ns,nr,irr,n", [(9, 21, 0.0, 130), (20, 60, 0.3, 200),
                                          (53, 325, 0.0, 333), (53, 325, 0.3, 129)])
def test_compiled_parity_both_layouts(torch, ak, ns, nr, irr, n):
    src, m = _mech(ak, ns, nr, irr)
    T, P, Y = synth.make_states(src, n, 5 + ns)
    Y[1, ::7] = 0.0          # the one-sided derivative at Y = 0
    Y[2, ::11] = -1e-9       # the clamp: a zero column
    nv = ns + 1
    for dt, tol in ((torch.float64, 1e-11), (torch.float32, 1e-6)):
        Tt, Pt, Yt = _dev(torch, dt, T, P, Y)
        J = ak.eval_jacobian(m, Tt, Pt, Yt)
        Ji = ak.eval_jacobian_interleaved(m, Tt, Pt, Yt)
        torch.cuda.synchronize()
        assert m.compiled_jacobian(dt)
        assert torch.equal(J.permute(1, 2, 0), Ji)
        Jn = J.cpu().numpy().astype(np.float64)
        if dt == torch.float64:
            _check(src, T, P, Y, Jn, tol)
        else:
            # the oracle on the float inputs the kernel saw
            T32, P32, Y32 = (a.astype(np.float32).astype(np.float64) for a in (T, P, Y))
            _check(src, T32, P32, Y32, Jn, tol)
        # the clamped column is zero in every species row
        assert np.all(Jn[::11, :ns, 2] == 0.0)


def test_compiled_bitwise_reproducible(torch, ak):
    src, m = _mech(ak, 53, 325)
    _, T, P, Y = synth.workload("c4", n_cells=4096)
    for dt in (torch.float64, torch.float32):
        Tt, Pt, Yt = _dev(torch, dt, T, P, Y)
        runs = [ak.eval_jacobian(m, Tt, Pt, Yt) for _ in range(3)]
        # the same cells at other positions of a larger batch (other lanes
        # and tiles): the values do not depend on them
        Tb, Pb, Yb = (torch.cat([a[..., :37], a], dim=-1).contiguous() for a in (Tt, Pt, Yt))
        Jb = ak.eval_jacobian(m, Tb, Pb, Yb)
        torch.cuda.synchronize()
        assert all(torch.equal(runs[0], r) for r in runs[1:])
        assert torch.equal(Jb[37:], runs[0]) and torch.equal(Jb[:37], runs[0][:37])


def test_compiled_matches_table_kernel(torch, ak):
    src, m = _mech(ak, 53, 325)
    _, T, P, Y = synth.workload("c4", n_cells=700)
    Tt, Pt, Yt = _dev(torch, torch.float64, T, P, Y)
    Jc = ak.eval_jacobian(m, Tt, Pt, Yt)
    os.environ["AK_JIT_JACOBIAN"] = "0"
    try:
        Jt = ak.eval_jacobian(m, Tt, Pt, Yt)
    finally:
        del os.environ["AK_JIT_JACOBIAN"]
    torch.cuda.synchronize()
    _, Ja = oracle.jacobian(src, T, P, Y, scales=True)
    d = np.abs(Jc.cpu().numpy() - Jt.cpu().numpy()) / np.maximum(Ja, 1e-300)
    assert float(d.max()) <= 2e-11


def test_compiled_strides_and_ragged_tile(torch, ak):
    src, m = _mech(ak, 20, 60, 0.3)
    n, nv = 77, 21
    T, P, Y = synth.make_states(src, n, 12)
    for dt in (torch.float64, torch.float32):
        Yw = torch.zeros((20, n + 9), dtype=dt, device="cuda")
        Yw[:, :n] = torch.tensor(Y, dtype=dt)
        Tt, Pt = _dev(torch, dt, T, P)
        ref = ak.eval_jacobian(m, Tt, Pt, Yw[:, :n].contiguous())
        # cell-major with a padded cell stride, Y with a padded row stride
        Jw = torch.full((n, nv * nv + 5), -7.0, dtype=dt, device="cuda")
        rc = ak.lib().ak_eval_jacobian(m.handle, ak._prec(dt), Tt.data_ptr(), Pt.data_ptr(),
                                       Yw.data_ptr(), n + 9, n, Jw.data_ptr(), nv * nv + 5, None)
        assert rc == 0
        # interleaved with a padded cell stride
        Ji = torch.full((nv * nv, n + 3), -7.0, dtype=dt, device="cuda")
        rc = ak.lib().ak_eval_jacobian_interleaved(m.handle, ak._prec(dt), Tt.data_ptr(),
                                                   Pt.data_ptr(), Yw.data_ptr(), n + 9, n,
                                                   Ji.data_ptr(), n + 3, None)
        assert rc == 0
        torch.cuda.synchronize()
        assert torch.equal(Jw[:, :nv * nv].reshape(n, nv, nv), ref)
        assert torch.equal(Ji[:, :n].reshape(nv, nv, n).permute(2, 0, 1), ref)
        assert bool((Jw[:, nv * nv:] == -7).all()) and bool((Ji[:, n:] == -7).all())


def test_compiled_bad_cells(torch, ak):
    src, m = _mech(ak, 9, 21)
    T, P, Y = synth.make_states(src, 70, 3)
    T[0], P[1], Y[2, 2], Y[:, 3] = -1.0, 0.0, np.nan, 0.0
    Tt, Pt, Yt = _dev(torch, torch.float64, T, P, Y)
    m.error_count()          # reads and clears the counter
    J = ak.eval_jacobian(m, Tt, Pt, Yt)
    Ji = ak.eval_jacobian_interleaved(m, Tt, Pt, Yt)
    torch.cuda.synchronize()
    Jn = J.cpu().numpy()
    assert all(np.all(np.isnan(Jn[i])) for i in range(4))
    assert np.all(np.isfinite(Jn[4:]))
    assert torch.equal(torch.nan_to_num(J.permute(1, 2, 0), nan=1.0),
                       torch.nan_to_num(Ji, nan=1.0))
    assert m.error_count() == 8


def test_interleaved_refuses(torch, ak):
    src = synth.with_pressure_dependence(synth.make_mechanism(9, 21), frac=0.5)
    m = ak.Mechanism(src)
    T, P, Y = synth.make_states(src, 8, 1)
    Tt, Pt, Yt = _dev(torch, torch.float64, T, P, Y)
    with pytest.raises(ak.AnnkinError) as e:
        ak.eval_jacobian_interleaved(m, Tt, Pt, Yt)
    assert e.value.code == -7
    big, mb = _mech(ak, 111, 784)
    T, P, Y = synth.make_states(big, 8, 1)
    Tt, Pt, Yt = _dev(torch, torch.float64, T, P, Y)
    with pytest.raises(ak.AnnkinError) as e:
        ak.eval_jacobian_interleaved(mb, Tt, Pt, Yt)
    assert e.value.code == -7
    assert not mb.compiled_jacobian(torch.float64)
    src9, m9 = _mech(ak, 9, 21)
    T, P, Y = synth.make_states(src9, 8, 1)
    Tt, Pt, Yt = _dev(torch, torch.float64, T, P, Y)
    out = torch.empty((10 * 10, 4), dtype=torch.float64, device="cuda")
    rc = ak.lib().ak_eval_jacobian_interleaved(m9.handle, ak._prec(torch.float64), Tt.data_ptr(),
                                               Pt.data_ptr(), Yt.data_ptr(), 8, 8,
                                               out.data_ptr(), 4, None)
    assert rc == -1      # ldJ < n_cells


def test_compiled_vjp_parity_and_bitwise(torch, ak):
    """The compiled VJP (gamma_j = sum_k g_k nu_kj, every reaction swept once
    per tile, waves' sums added in a fixed order) against J^T g from the
    oracle's Jacobian, bitwise under repetition and batch position, and
    against the table-driven kernel."""
    for ns, nr, irr in ((9, 21, 0.0), (53, 325, 0.3)):
        src, m = _mech(ak, ns, nr, irr)
        n = 157
        T, P, Y = synth.make_states(src, n, 40 + ns)
        Y[3, ::5] = -1e-9
        g = np.random.default_rng(ns).standard_normal((ns, n))
        for dt, tol in ((torch.float64, 1e-11), (torch.float32, 1e-6)):
            Tt, Pt, Yt, gt = _dev(torch, dt, T, P, Y, g)
            gY, gT = ak.eval_vjp(m, Tt, Pt, Yt, gt)
            gY2, gT2 = ak.eval_vjp(m, Tt, Pt, Yt, gt)
            Tb, Pb, Yb, gb = (torch.cat([a[..., :21], a], dim=-1).contiguous()
                              for a in (Tt, Pt, Yt, gt))
            gYb, gTb = ak.eval_vjp(m, Tb, Pb, Yb, gb)
            os.environ["AK_JIT_VJP"] = "0"
            try:
                gYt, gTt = ak.eval_vjp(m, Tt, Pt, Yt, gt)
            finally:
                del os.environ["AK_JIT_VJP"]
            torch.cuda.synchronize()
            assert torch.equal(gY, gY2) and torch.equal(gT, gT2)
            assert torch.equal(gYb[:, 21:], gY) and torch.equal(gTb[21:], gT)
            if dt == torch.float32:
                Tc, Pc, Yc, gc = (a.astype(np.float32).astype(np.float64) for a in (T, P, Y, g))
            else:
                Tc, Pc, Yc, gc = T, P, Y, g
            Jr, Ja = oracle.jacobian(src, Tc, Pc, Yc, precision="ld", scales=True)
            ref = np.einsum("ki,ikc->ci", gc, Jr[:, :ns, :].astype(np.float64))
            scale = np.einsum("ki,ikc->ci", np.abs(gc), Ja[:, :ns, :].astype(np.float64))
            got = np.vstack([gY.cpu().numpy().astype(np.float64),
                             gT.cpu().numpy().astype(np.float64)[None, :]])
            tab = np.vstack([gYt.cpu().numpy().astype(np.float64),
                             gTt.cpu().numpy().astype(np.float64)[None, :]])
            e = np.abs(got - ref) / np.maximum(scale, 1e-300)
            print("vjp", ns, nr, dt, "max err/scale", float(e.max()), flush=True)
            assert float(e.max()) <= tol
            assert float((np.abs(got - tab) / np.maximum(scale, 1e-300)).max()) <= 2 * tol
            # the clamped species' adjoint is zero
            assert np.all(got[3, ::5] == 0.0)
