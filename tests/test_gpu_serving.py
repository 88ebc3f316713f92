"""GPU tests of the serving loop: results in a mixed, concurrent request
stream equal each request evaluated alone (ak_eval_source) -- bitwise where
the mechanism has compiled kernels, which run the same code in both, within
rounding of the omega accumulation for the table-driven kernels -- and match
the oracle; memory-based admission, cancellation, shutdown and statistics."""

import threading

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


@pytest.fixture(scope="module")
def mechs(ak):
    out = {}
    for ns, nr in ((9, 21), (53, 325)):
        src = synth.make_mechanism(ns, nr)
        out[ns] = (src, ak.Mechanism(src))
    return out


def _request_states(src, n, seed, dtype):
    T, P, Y = synth.make_states(src, n, seed, (800.0, 2800.0), (1.0, 20.0), 0.3, dtype=dtype)
    return T, P, Y


def _pinned(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).pin_memory()


def _alone(torch, ak, m, T, P, Y):
    Tt, Pt, Yt = (torch.tensor(a, device="cuda") for a in (T, P, Y))
    om = ak.eval_source(m, Tt, Pt, Yt)
    torch.cuda.synchronize()
    return om.cpu().numpy()


@pytest.mark.parametrize("batching", [True, False])
def test_mixed_concurrent_stream_equals_alone(torch, ak, mechs, batching):
    srv = ak.Server(max_inflight=3, batching=batching, arena_bytes=256 << 20)
    rng = np.random.default_rng(3)
    specs = []
    for i in range(60):
        ns = 9 if rng.random() < 0.5 else 53
        dt = np.float32 if rng.random() < 0.7 else np.float64
        n = int(np.round(np.exp(rng.uniform(np.log(64), np.log(6000)))))
        specs.append((i, ns, dt, n))
    results = {}
    lock = threading.Lock()

    def client(part):
        for i, ns, dt, n in part:
            src, m = mechs[ns]
            T, P, Y = _request_states(src, n, 500 + i, dt)
            # Y inside a wider buffer: a strided host leading dimension
            Yb = np.zeros((ns, n + 7), dtype=dt)
            Yb[:, :n] = Y
            Tp, Pp, Yp = _pinned(torch, T), _pinned(torch, P), _pinned(torch, Yb)
            out = torch.zeros((ns, n), dtype=torch.float32 if dt == np.float32 else torch.float64).pin_memory()
            req = srv.submit(m, Tp, Pp, Yp[:, :n], out)
            req.wait(60.0)
            req.free()
            with lock:
                results[i] = (T, P, Y, out.numpy().copy())

    threads = [threading.Thread(target=client, args=(specs[k::4],)) for k in range(4)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert len(results) == len(specs)
    st = srv.stats()
    print("server stats", st, flush=True)
    assert st["completed"] == len(specs) and st["failed"] == 0
    assert st["p99_ms"] >= st["p50_ms"] > 0 and st["cells_per_s"] > 0
    if not batching:
        assert st["batches"] == len(specs)
    srv.close()
    for i, ns, dt, n in specs:
        src, m = mechs[ns]
        T, P, Y, om = results[i]
        alone = _alone(torch, ak, m, T, P, Y)
        _, S, _ = oracle.source(src, T.astype(np.float64), P.astype(np.float64),
                                Y.astype(np.float64), scales=True)
        if m.compiled(dt):
            # the same compiled kernel, fixed accumulation order: bitwise
            assert np.array_equal(om, alone), i
        elif dt == np.float32:
            assert np.all(np.abs(om.astype(np.float64) - alone) <= 1e-6 * S), i
        else:
            assert np.all(np.abs(om - alone) <= 1e-13 * S), i
        ref = oracle.source(src, T.astype(np.float64), P.astype(np.float64), Y.astype(np.float64))
        tol = 1e-5 if dt == np.float32 else 1e-12
        assert np.all(np.abs(om.astype(np.float64) - ref) <= tol * S), i


def test_continuous_batching_fuses_requests(torch, ak, mechs):
    """Requests queued while a batch runs are admitted together: fewer
    batches than requests."""
    src, m = mechs[53]
    srv = ak.Server(max_inflight=1, batching=True, arena_bytes=512 << 20)
    T, P, Y = _request_states(src, 4000, 77, np.float32)
    Tp, Pp, Yp = _pinned(torch, T), _pinned(torch, P), _pinned(torch, Y)
    outs = [torch.zeros((53, 4000), dtype=torch.float32).pin_memory() for _ in range(40)]
    reqs = [srv.submit(m, Tp, Pp, Yp, o) for o in outs]
    for r in reqs:
        r.wait(60.0)
        r.free()
    st = srv.stats()
    print("stats", st, flush=True)
    assert st["completed"] == 40
    assert st["batches"] < 40
    assert st["launches"] == st["batches"]          # one launch per batch (one mechanism, FP32)
    alone = _alone(torch, ak, m, T, P, Y)
    assert m.compiled(np.float32)
    for o in outs:
        assert np.array_equal(o.numpy(), alone)
    srv.close()


def test_admission_limits_and_errors(torch, ak, mechs):
    src, m = mechs[53]
    srv = ak.Server(max_inflight=1, arena_bytes=4 << 20)
    T, P, Y = _request_states(src, 20000, 5, np.float32)     # ~8.6 MB > arena
    out = np.zeros((53, 20000), np.float32)
    with pytest.raises(ak.AnnkinError) as e:
        srv.submit(m, T, P, Y, out)
    assert e.value.code == -4
    # requests that each fit but not together are serialised by memory
    T2, P2, Y2 = _request_states(src, 6000, 6, np.float32)   # ~2.6 MB each
    outs = [np.zeros((53, 6000), np.float32) for _ in range(3)]
    reqs = [srv.submit(m, T2, P2, Y2, o) for o in outs]
    for r in reqs:
        r.wait(60.0)
        r.free()
    alone = _alone(torch, ak, m, T2, P2, Y2)
    for o in outs:
        assert np.array_equal(o, alone)
    assert srv.stats()["arena_used"] == 0
    srv.close()


def test_cancel_and_shutdown(torch, ak, mechs):
    src, m = mechs[53]
    srv = ak.Server(max_inflight=1, batching=False)
    T, P, Y = _request_states(src, 30000, 8, np.float32)
    outs = [np.zeros((53, 30000), np.float32) for _ in range(12)]
    reqs = [srv.submit(m, T, P, Y, o) for o in outs]
    cancelled = [r.cancel() for r in reqs[::-1]][::-1]
    assert any(cancelled)                       # the tail was still queued
    for r, c in zip(reqs, cancelled):
        if c:
            with pytest.raises(ak.AnnkinError) as e:
                r.wait(10.0)
            assert e.value.code == -6
        else:
            r.wait(60.0)
        r.free()
    # shutdown with queued work: queued requests are cancelled, admitted drain
    more = [srv.submit(m, T, P, Y, o) for o in outs[:6]]
    srv.close()
    codes = []
    for r in more:
        try:
            r.wait(10.0)
            codes.append(0)
        except ak.AnnkinError as e:
            codes.append(e.code)
        r.free()
    assert set(codes) <= {0, -6}


def test_mix_with_large_mechanisms(torch, ak, mechs):
    """One batch mixing a compiled mechanism with the table-driven kernels of
    larger ones (111 and 140 species: the fused launch then runs the
    instantiation sized for the largest), against the oracle and alone."""
    big = {}
    for ns, nr, seed in ((111, 784, 2), (140, 520, 7)):
        src = synth.make_mechanism(ns, nr, seed=seed)
        big[ns] = (src, ak.Mechanism(src))
    allm = {9: mechs[9], **big}
    srv = ak.Server(max_inflight=1, batching=True, arena_bytes=256 << 20)
    specs = [(0, 9, 300), (1, 111, 700), (2, 140, 500), (3, 9, 64), (4, 140, 129),
             (5, 111, 65)]
    reqs, bufs = [], {}
    for i, ns, n in specs:
        src, m = allm[ns]
        T, P, Y = _request_states(src, n, 900 + i, np.float32)
        out = torch.zeros((ns, n), dtype=torch.float32).pin_memory()
        bufs[i] = (T, P, Y, out)
        reqs.append(srv.submit(m, _pinned(torch, T), _pinned(torch, P), _pinned(torch, Y),
                               out))
    for r in reqs:
        r.wait(60.0)
        r.free()
    assert srv.stats()["batches"] < len(specs)
    srv.close()
    for i, ns, n in specs:
        src, m = allm[ns]
        T, P, Y, out = bufs[i]
        om = out.numpy().astype(np.float64)
        T64, P64, Y64 = (a.astype(np.float64) for a in (T, P, Y))
        ref, S, _ = oracle.source(src, T64, P64, Y64, scales=True)
        assert np.all(np.abs(om - ref) <= 1e-5 * S), (i, ns)
        alone = _alone(torch, ak, m, T, P, Y).astype(np.float64)
        if m.compiled(np.float32):
            assert np.array_equal(om, alone), i
        else:
            assert np.all(np.abs(om - alone) <= 1e-6 * S), (i, ns)
    for _, m in big.values():
        m.close()


def test_caller_provided_arena(torch, ak, mechs):
    """The server stages requests in a device buffer the caller owns: results
    bitwise as alone, the arena's size in the statistics, the buffer left to
    the caller after the server is gone; bad buffers are refused."""
    arena = torch.empty(32 << 20, dtype=torch.uint8, device="cuda")
    srv = ak.Server(max_inflight=2, batching=True, arena=arena)
    assert srv.stats()["arena_bytes"] == 32 << 20
    reqs = []
    for i, (ns, n) in enumerate(((53, 1000), (9, 70), (53, 5000), (9, 3000))):
        src, m = mechs[ns]
        T, P, Y = _request_states(src, n, 700 + i, np.float32)
        out = torch.zeros(Y.shape, dtype=torch.float32).pin_memory()
        pins = [_pinned(torch, a) for a in (T, P, Y)]
        reqs.append((srv.submit(m, *pins, out), m, (T, P, Y), out, pins))
    for r, *_ in reqs:
        r.wait(60.0)
        r.free()
    srv.close()
    for _, m, (T, P, Y), out, _ in reqs:
        assert np.array_equal(out.numpy(), _alone(torch, ak, m, T, P, Y))
    arena.fill_(1)                       # still the caller's, usable
    torch.cuda.synchronize()
    with pytest.raises(ValueError):
        ak.Server(arena=torch.empty(1 << 20, dtype=torch.uint8))       # host memory
    with pytest.raises(ak.AnnkinError) as e:
        ak.Server(arena=arena[1:])                                     # not aligned
    assert e.value.code == -1
