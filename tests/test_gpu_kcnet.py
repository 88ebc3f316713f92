"""GPU parity of the ln K_c layer and its trained replacement (Sec. 2.3)
against the oracle, through the C ABI:
  - ak_eval_lnkc (Gibbs and stoichiometric layers, Eqs. 9-11) against the
    oracle's ln K_c (Eq. 8);
  - ak_eval_lnkc_net (Architecture 2) against the oracle's float64 network
    on the same weights, within a rounding bound derived from the arithmetic:
    |d| <= c u (N_H (N_L + 1) + 8) m, with u the unit roundoff of the path,
    m the oracle's running magnitude of the same computation and c = 4;
  - ak_eval_source_lnkc against the oracle's source term with the same given
    ln K_c, |d omega| <= tol S (S the gross rate scale), tol 1e-12 (FP64)
    and 1e-6 (FP32, inputs rounded to float on both sides);
  - ak_eval_source_net against the oracle's source term fed by the oracle's
    network: the FP32 network error of ln K_c enters q_r as a relative
    error, so tol = 1e-6 + 1.1 max |d ln K_c bound|.
Weights are seeded random (parity needs no training); sizes span several
tiles with ragged ends, padded widths (12 -> 16, 40 -> 64) and bad cells.
"""

import numpy as np
import pytest

import oracle
from paper_2008_08483_amd import kcnet, synth

pytestmark = pytest.mark.gpu

U = {"f64": 2.0 ** -53, "f32": 2.0 ** -24}


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


def _mech(ak, ns, nr, irrev=0.0):
    key = (ns, nr, irrev)
    if key not in _M:
        src = synth.make_mechanism(ns, nr)
        if irrev:
            rng = np.random.default_rng(5)
            src.reversible = (rng.random(nr) >= irrev).astype(np.uint8)
        _M[key] = (src, ak.Mechanism(src))
    return _M[key]


def _dt(torch, prec):
    return torch.float64 if prec == "f64" else torch.float32


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("ns,nr,n", [(9, 21, 1000), (53, 325, 4099)])
def test_lnkc_exact(torch, ak, prec, ns, nr, n):
    src, m = _mech(ak, ns, nr)
    rng = np.random.default_rng(ns)
    T = rng.uniform(300.0, 3500.0, n)
    T[:4] = [999.9999, 1000.0, 1000.0000001, 300.0]   # both NASA ranges near T_mid
    dt = _dt(torch, prec)
    Tg = torch.tensor(T, dtype=dt, device="cuda")
    Tx = Tg.double().cpu().numpy()                    # what the kernel sees
    out = torch.full((nr, n + 5), 7.0, dtype=dt, device="cuda")
    ak.eval_lnkc(m, Tg, out=out[:, :n])
    got = out.cpu().numpy().astype(np.float64)
    ref = oracle.lnkc(src, Tx, precision="ld").astype(np.float64)
    # double arithmetic from weights folded at load time: a few ulps of the
    # terms' sizes; FP32 adds the rounding of the result
    tol = 1e-11 * (1.0 + np.abs(ref)) + (U[prec] * 2 * np.abs(ref) if prec == "f32" else 0)
    assert np.all(np.abs(got[:, :n] - ref) <= tol)
    assert np.all(got[:, n:] == 7.0)                  # padding untouched


def test_lnkc_bad_cells(torch, ak):
    src, m = _mech(ak, 9, 21)
    m.error_count()
    T = torch.tensor([1500.0, float("nan"), -3.0, 0.0, 800.0], dtype=torch.float64, device="cuda")
    out = ak.eval_lnkc(m, T).cpu().numpy()
    assert np.all(np.isnan(out[:, 1:4])) and np.all(np.isfinite(out[:, [0, 4]]))
    assert m.error_count() == 3


def _bound(net, T, prec):
    ref, mag = oracle.kcnet(net, T, bound=True)
    c = 4.0 * U[prec] * (net.n_hidden * (net.n_layers + 1) + 8)
    return ref, c * mag


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("layers,hidden,nr,n", [(1, 8, 21, 1000), (2, 12, 21, 777),
                                                (3, 32, 325, 4099), (2, 40, 60, 513),
                                                (1, 64, 325, 300)])
def test_kcnet_parity(torch, ak, prec, layers, hidden, nr, n):
    net_w = kcnet.random_weights(layers, hidden, nr, seed=layers * 100 + hidden)
    net = ak.KcNet(net_w)
    rng = np.random.default_rng(hidden)
    dt = _dt(torch, prec)
    Tg = torch.tensor(rng.uniform(250.0, 6000.0, n), dtype=dt, device="cuda")
    Tx = Tg.double().cpu().numpy()
    out = torch.full((nr, n + 3), 5.0, dtype=dt, device="cuda")
    ak.eval_lnkc_net(net, Tg, out=out[:, :n])
    got = out.cpu().numpy().astype(np.float64)
    ref, bound = _bound(net_w, Tx, prec)
    assert np.all(np.abs(got[:, :n] - ref) <= bound)
    assert np.all(got[:, n:] == 5.0)
    # fixed summation order: a second call is bitwise equal
    again = ak.eval_lnkc_net(net, Tg)
    assert torch.equal(again, out[:, :n])


def test_kcnet_bad_cells_and_refusals(torch, ak):
    net_w = kcnet.random_weights(1, 8, 5, seed=1)
    net = ak.KcNet(net_w)
    T = torch.tensor([1500.0, float("inf"), -1.0, 600.0], dtype=torch.float32, device="cuda")
    out = ak.eval_lnkc_net(net, T).cpu().numpy()
    assert np.all(np.isnan(out[:, 1:3])) and np.all(np.isfinite(out[:, [0, 3]]))
    bad = kcnet.random_weights(1, 65, 5, seed=1)       # wider than the kernels hold
    with pytest.raises(ak.AnnkinError) as e:
        ak.KcNet(bad)
    assert e.value.code == -1
    nanw = kcnet.random_weights(1, 8, 5, seed=1)
    nanw.weights[1][0, 0] = np.nan
    with pytest.raises(ak.AnnkinError):
        ak.KcNet(nanw)


def _states(src, n, seed, torch, dt):
    T, P, Y = synth.make_states(src, n, seed, (800.0, 2800.0), (1.0, 20.0), 0.3)
    Y[3, :7] = 0.0          # a species absent from some cells
    Y[1, 5] = -1e-6         # and a slightly negative mass fraction
    g = [torch.tensor(a, dtype=dt, device="cuda") for a in (T, P, Y)]
    return g, [a.double().cpu().numpy() for a in g]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("ns,nr,irrev,n", [(9, 21, 0.0, 1000), (53, 325, 0.3, 2053)])
def test_source_with_given_lnkc(torch, ak, prec, ns, nr, irrev, n):
    src, m = _mech(ak, ns, nr, irrev)
    dt = _dt(torch, prec)
    (Tg, Pg, Yg), (T, P, Y) = _states(src, n, 21, torch, dt)
    # exact ln K_c shifted by up to +-2: q_r no longer balances q_f anywhere
    rng = np.random.default_rng(3)
    K = oracle.lnkc(src, T) + rng.uniform(-2.0, 2.0, (nr, n))
    Kg = torch.tensor(K, dtype=dt, device="cuda")
    Kx = Kg.double().cpu().numpy()
    out = torch.full((ns, n + 2), 3.0, dtype=dt, device="cuda")
    ak.eval_source_lnkc(m, Tg, Pg, Yg, Kg, out=out[:, :n])
    got = out.cpu().numpy().astype(np.float64)
    ref, S, _ = oracle.source_lnkc(src, T, P, Y, Kx, precision="ld", scales=True)
    ref, S = ref.astype(np.float64), S.astype(np.float64)
    tol = 1e-12 if prec == "f64" else 1e-6
    assert np.all(np.abs(got[:, :n] - ref) <= tol * S + 1e-300)
    assert np.all(got[:, n:] == 3.0)
    again = ak.eval_source_lnkc(m, Tg, Pg, Yg, Kg)
    assert torch.equal(again, out[:, :n])


def test_source_with_exact_lnkc_matches_the_source(torch, ak):
    # the exact ln K_c fed back reproduces the compiled source term
    src, m = _mech(ak, 53, 325)
    (Tg, Pg, Yg), (T, P, Y) = _states(src, 1500, 22, torch, torch.float64)
    om = ak.eval_source_lnkc(m, Tg, Pg, Yg, ak.eval_lnkc(m, Tg)).cpu().numpy()
    ref = ak.eval_source(m, Tg, Pg, Yg).cpu().numpy()
    _, S, _ = oracle.source(src, T, P, Y, scales=True)
    assert np.all(np.abs(om - ref) <= 1e-12 * S)


@pytest.fixture(scope="module")
def trained_53(ak):
    # a 3/32 network fitted (on the CPU) to the oracle's ln K_c over the
    # states' temperature range, so that its q_r stay near the true ones
    src, _ = _mech(ak, 53, 325)
    T = np.random.default_rng(8).uniform(800.0, 2800.0, 20000)
    return kcnet.train(T, oracle.lnkc(src, T), 3, 32, epochs=30, batch=1024, seed=2)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_source_net(torch, ak, prec, trained_53):
    src, m = _mech(ak, 53, 325)
    net_w = trained_53
    net = ak.KcNet(net_w)
    dt = _dt(torch, prec)
    (Tg, Pg, Yg), (T, P, Y) = _states(src, 3001, 23, torch, dt)
    got = ak.eval_source_net(m, net, Tg, Pg, Yg).cpu().numpy().astype(np.float64)
    K, kb = _bound(net_w, T, prec)
    ref, S, _ = oracle.source_lnkc(src, T, P, Y, K, scales=True)
    tol = (1e-12 if prec == "f64" else 1e-6) + 1.1 * kb.max()
    assert np.all(np.abs(got - ref) <= tol * S + 1e-300)
    # the same as the two calls in sequence, bitwise
    two = ak.eval_source_lnkc(m, Tg, Pg, Yg, ak.eval_lnkc_net(net, Tg))
    assert np.array_equal(two.cpu().numpy().astype(np.float64), got)


def test_source_net_refusals(torch, ak):
    src, m = _mech(ak, 9, 21)
    net = ak.KcNet(kcnet.random_weights(1, 8, 20, seed=4))      # 20 outputs, 21 reactions
    (Tg, Pg, Yg), _ = _states(src, 64, 24, torch, torch.float64)
    with pytest.raises(ak.AnnkinError) as e:
        ak.eval_source_net(m, net, Tg, Pg, Yg)
    assert e.value.code == -1
    pd = synth.with_pressure_dependence(synth.make_mechanism(9, 21), frac=0.5)
    mp_ = ak.Mechanism(pd)
    with pytest.raises(ak.AnnkinError) as e:
        ak.eval_source_lnkc(mp_, Tg, Pg, Yg, ak.eval_lnkc(mp_, Tg))
    assert e.value.code == -7


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("pattern", ["two", "distinct"])
def test_lnkc_exact_mixed_tmid(torch, ak, prec, pattern):
    # per-species T_mid: two values (up to 3 intervals per reaction, the
    # composed layers) or all distinct (up to 5 intervals: the layers run
    # separately); temperatures include every T_mid exactly
    src = synth.make_mechanism(20, 60)
    rng = np.random.default_rng(11)
    if pattern == "two":
        src.T_mid = np.where(rng.random(20) < 0.5, 1000.0, 1300.0)
    else:
        src.T_mid = rng.uniform(700.0, 1500.0, 20).round(3)
    m = ak.Mechanism(src)
    n = 700
    T = rng.uniform(300.0, 3000.0, n)
    T[:20] = src.T_mid
    T[20:40] = np.nextafter(src.T_mid, 0.0)
    dt = _dt(torch, prec)
    Tg = torch.tensor(T, dtype=dt, device="cuda")
    Tx = Tg.double().cpu().numpy()
    got = ak.eval_lnkc(m, Tg).cpu().numpy().astype(np.float64)
    ref = oracle.lnkc(src, Tx, precision="ld").astype(np.float64)
    tol = 1e-11 * (1.0 + np.abs(ref)) + (U[prec] * 2 * np.abs(ref) if prec == "f32" else 0)
    assert np.all(np.abs(got - ref) <= tol)
    m.close()


def test_empty_batches_and_argument_errors(torch, ak):
    src, m = _mech(ak, 9, 21)
    net = ak.KcNet(kcnet.random_weights(1, 8, 21, seed=5))
    e64 = torch.empty(0, dtype=torch.float64, device="cuda")
    assert ak.eval_lnkc(m, e64).shape == (21, 0)
    assert ak.eval_lnkc_net(net, e64).shape == (21, 0)
    Y0 = torch.empty((9, 0), dtype=torch.float64, device="cuda")
    assert ak.eval_source_net(m, net, e64, e64, Y0).shape == (9, 0)
    T = torch.full((5,), 1200.0, dtype=torch.float64, device="cuda")
    lib = ak.lib()
    out = torch.empty((21, 5), dtype=torch.float64, device="cuda")
    # ldK below n, null pointers, bad precision: refused before any launch
    assert lib.ak_eval_lnkc(m.handle, 0, T.data_ptr(), 5, out.data_ptr(), 4, None) == -1
    assert lib.ak_eval_lnkc(m.handle, 0, None, 5, out.data_ptr(), 5, None) == -1
    assert lib.ak_eval_lnkc(m.handle, 7, T.data_ptr(), 5, out.data_ptr(), 5, None) == -1
    assert lib.ak_eval_lnkc_net(net.handle, 0, T.data_ptr(), 5, out.data_ptr(), 4, None) == -1
    assert lib.ak_eval_lnkc_net(None, 0, T.data_ptr(), 5, out.data_ptr(), 5, None) == -1
    assert lib.ak_eval_source_lnkc(m.handle, 0, T.data_ptr(), T.data_ptr(), None, 5, 5,
                                   out.data_ptr(), 5, out.data_ptr(), 5, None) == -1
    assert (out.isnan() | out.isfinite()).all()


@pytest.mark.parametrize("ns,nr,dt", [(9, 21, 1e-14), (53, 325, 5e-16)])
def test_integrate_euler_with_network(torch, ak, ns, nr, dt):
    # the 0-D reactor driven by a trained network's ln K_c (Sec. 3.1's
    # a-posteriori use) against the oracle's composition with the same
    # network; FP64, 30 steps
    mild = dict(ln_A_range=(8.0, 16.0), Ea_range=(20000.0, 60000.0))
    src = synth.make_mechanism(ns, nr, **mild)
    m = ak.Mechanism(src)
    Ttr = np.random.default_rng(13).uniform(900.0, 2700.0, 8000)
    w = kcnet.train(Ttr, oracle.lnkc(src, Ttr), 1, 16, epochs=15, batch=512, lr=1e-2, seed=3)
    net = ak.KcNet(w)
    T, P, Y = synth.make_states(src, 70, 31, (1000.0, 2500.0), (1.0, 20.0), 0.5)
    Tt, Pt, Yt = (torch.tensor(a, dtype=torch.float64, device="cuda") for a in (T, P, Y))
    ak.integrate_euler_net(m, net, Tt, Pt, Yt, dt, 30)
    torch.cuda.synchronize()
    T1, Y1 = oracle.integrate_euler_lnkc(src, lambda t: oracle.kcnet(w, t), T, P, Y, dt, 30)
    assert np.abs(T1 - T).max() > 0.1
    np.testing.assert_allclose(Tt.cpu().numpy(), T1, rtol=1e-11, atol=0)
    assert np.abs(Yt.cpu().numpy() - Y1).max() <= 1e-11 * Y.sum(axis=0).max()
    # and the exact integrator, for scale: the network's error in ln K_c moves
    # the trajectory by far more than rounding
    Te, Ye = (torch.tensor(a, dtype=torch.float64, device="cuda") for a in (T, Y))
    ak.integrate_euler(m, Te, Pt, Ye, dt, 30)
    torch.cuda.synchronize()
    print("ann vs exact after 30 steps: max |dT| %.3e K, max |dY| %.3e" % (
        np.abs(Te.cpu().numpy() - T1).max(), np.abs(Ye.cpu().numpy() - Y1).max()))
    m.close()
