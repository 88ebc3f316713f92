"""Training of the approximate ln K_c network (Sec. 2.3, Architecture 2) on
the CPU, on targets from the oracle's ln K_c: the loss falls, the exported
weights evaluated by the oracle's network reproduce the trained fit (so the
export keeps the X W orientation and the standardization), and the weights
survive a save/load round trip."""

import numpy as np
import pytest

import oracle
from paper_2008_08483_amd import kcnet, synth


@pytest.fixture(scope="module")
def data():
    mech = synth.make_mechanism(9, 21)
    rng = np.random.default_rng(0)
    T = rng.uniform(300.0, 3000.0, 20000)
    return mech, T, oracle.lnkc(mech, T)


@pytest.mark.parametrize("layers,hidden,epochs,batch,lr,goal", [(1, 8, 60, 256, 1e-2, 0.03),
                                                                (3, 32, 40, 1024, 3e-3, 0.02)])
def test_training_fits_lnkc(data, layers, hidden, epochs, batch, lr, goal):
    mech, T, K = data
    net = kcnet.train(T, K, layers, hidden, epochs=epochs, batch=batch, lr=lr, seed=1)
    assert net.n_layers == layers and net.n_hidden == hidden and net.n_out == mech.n_reactions
    assert net.history[-1] < 0.2 * net.history[0]
    # the exported weights, evaluated in float64 by the oracle's network,
    # give the standardized error the training reached
    pred = oracle.kcnet(net, T)
    mse = np.mean(((pred - K) / net.y_std[:, None]) ** 2)
    assert mse < 2.0 * net.history[-1] + 1e-6
    assert mse < goal


def test_random_weights_shapes():
    net = kcnet.random_weights(3, 32, 325, seed=2)
    assert [w.shape for w in net.weights] == [(1, 32), (32, 32), (32, 32), (32, 325)]
    assert [b.shape for b in net.biases] == [(32,), (32,), (32,), (325,)]
    assert net.y_mean.shape == (325,) and np.all(net.y_std > 0)


def test_save_load_round_trip(tmp_path, data):
    mech, T, K = data
    net = kcnet.train(T[:2000], K[:, :2000], 1, 8, epochs=2, batch=512, seed=3)
    p = str(tmp_path / "net.npz")
    net.save(p)
    back = kcnet.KcNetWeights.load(p)
    for a, b in zip(net.weights + net.biases, back.weights + back.biases):
        assert np.array_equal(a, b)
    assert back.x_mean == net.x_mean and back.x_std == net.x_std
    assert np.array_equal(back.y_mean, net.y_mean) and np.array_equal(back.y_std, net.y_std)
    np.testing.assert_array_equal(oracle.kcnet(back, T[:50]), oracle.kcnet(net, T[:50]))
