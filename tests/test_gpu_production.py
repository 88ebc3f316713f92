"""GPU parity of ak_eval_production, the stoichiometric contraction
omega = nu r (Eq. 2) of given FP32 rates of progress on the matrix cores in
split bfloat16, against the oracle's float64 product nu r of the same FP32
rates.  nu is exact in bfloat16 and each rate splits exactly into three
bfloat16 parts, so every product is exact and the only error is FP32
accumulation over 3 N_R terms; the bound is the classical one for a sum in
any order, |d omega_k| <= (3 N_R + 2) u sum_j |nu_kj| |r_j| with u = 2^-24,
plus 1e-30 for rates whose lowest part falls below the normal range.
Integer rates of small magnitude make every partial sum exact: there the
result must equal the oracle bit for bit.  Cases span one to several
species groups (16 species per MFMA block, 8 blocks per workgroup), ragged
reaction chunks (32 per step), ragged cell tiles, strided buffers, the
empty batch, and sampled cells at 53/325 x 2^20."""

import ctypes as C

import numpy as np
import pytest

import oracle
from paper_2008_08483_amd import synth

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.fixture(scope="module")
def ak():
    from paper_2008_08483_amd import annkin
    return annkin


_M = {}


def _mech(ak, ns, nr):
    if (ns, nr) not in _M:
        src = synth.make_mechanism(ns, nr)
        _M[(ns, nr)] = (src, ak.Mechanism(src))
    return _M[(ns, nr)]


def _rates(nr, n, seed):
    rng = np.random.default_rng(seed)
    mag = 10.0 ** rng.uniform(-20.0, 10.0, (nr, n))
    return (rng.standard_normal((nr, n)) * mag).astype(np.float32)


def _bound(src, r):
    absnu = np.abs(src.nu_r.astype(float) - src.nu_f.astype(float)).T
    return (3 * src.nu_f.shape[0] + 2) * U32 * (absnu @ np.abs(r.astype(np.float64))) + 1e-30


@pytest.mark.parametrize("ns,nr,n,seed", [(9, 21, 1, 1), (9, 21, 77, 2), (53, 325, 1000, 3),
                                          (53, 325, 4099, 4), (150, 600, 515, 5)])
def test_production_parity(torch, ak, ns, nr, n, seed):
    src, mech = _mech(ak, ns, nr)
    r = _rates(nr, n, seed)
    want = oracle.production(src, r)
    got = ak.eval_production(mech, torch.from_numpy(r).cuda()).cpu().numpy()
    torch.cuda.synchronize()
    d = np.abs(got.astype(np.float64) - want)
    assert np.all(d <= _bound(src, r)), (d / _bound(src, r)).max()


@pytest.mark.parametrize("ns,nr", [(9, 21), (53, 325), (150, 600)])
def test_integer_rates_are_exact(torch, ak, ns, nr):
    src, mech = _mech(ak, ns, nr)
    rng = np.random.default_rng(11)
    r = rng.integers(-2000, 2001, (nr, 333)).astype(np.float32)
    got = ak.eval_production(mech, torch.from_numpy(r).cuda()).cpu().numpy()
    np.testing.assert_array_equal(got.astype(np.float64), oracle.production(src, r))


def test_strided_buffers_and_repeatability(torch, ak):
    src, mech = _mech(ak, 53, 325)
    n, ld = 700, 1024
    r = _rates(325, n, 7)
    buf = torch.full((325, ld), float("nan"), dtype=torch.float32, device="cuda")
    buf[:, :n] = torch.from_numpy(r).cuda()
    out = torch.full((53, ld), -7.0, dtype=torch.float32, device="cuda")
    a = ak.eval_production(mech, buf[:, :n], out=out[:, :n]).clone()
    b = ak.eval_production(mech, buf[:, :n])
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert torch.all(out[:, n:] == -7.0)            # nothing written past n_cells
    d = np.abs(a.cpu().numpy().astype(np.float64) - oracle.production(src, r))
    assert np.all(d <= _bound(src, r))


def test_empty_batch_and_errors(torch, ak):
    src, mech = _mech(ak, 9, 21)
    out = ak.eval_production(mech, torch.zeros((21, 0), dtype=torch.float32, device="cuda"))
    assert out.shape == (9, 0)
    lib = ak.lib()
    r = torch.zeros((21, 8), dtype=torch.float32, device="cuda")
    o = torch.zeros((9, 8), dtype=torch.float32, device="cuda")
    assert lib.ak_eval_production(mech.handle, C.c_void_p(r.data_ptr()), 4, 8,
                                  C.c_void_p(o.data_ptr()), 8, None) == -1
    assert b"ldR" in lib.ak_last_error()
    assert lib.ak_eval_production(mech.handle, None, 8, 8, C.c_void_p(o.data_ptr()), 8,
                                  None) == -1
    with pytest.raises(ValueError):
        ak.eval_production(mech, r.double())


def test_full_size_sampled(torch, ak):
    # the forward bench's workload shape: 53/325 x 2^20 cells, checked on
    # 4096 sampled cells
    src, mech = _mech(ak, 53, 325)
    n = 1 << 20
    g = torch.Generator(device="cuda").manual_seed(9)
    r = torch.randn((325, n), generator=g, device="cuda", dtype=torch.float32)
    r *= torch.pow(10.0, torch.empty_like(r).uniform_(-20.0, 10.0, generator=g))
    out = ak.eval_production(mech, r)
    idx = np.random.default_rng(3).choice(n, 4096, replace=False)
    it = torch.from_numpy(idx).cuda()
    rs = r[:, it].cpu().numpy()
    got = out[:, it].cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - oracle.production(src, rs)) <= _bound(src, rs))
