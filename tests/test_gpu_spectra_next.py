"""Orientation-resolved Raman map, Raman prefactor and streaming correlation
accumulators on the GPU against the FP64 oracle (direct lag sums).

Bound: per spectrum max_k |S_gpu - S_ref| / max_k |S_ref| <= 1e-4
(tests/parity.py); the GPU reaches the correlations through zero-padded FFTs,
the oracle through direct sums.
"""
import numpy as np
import pytest

import oracle
from parity import SPECTRUM_TOL, spectrum_error

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = gpu_lib.Context(0)
    yield c
    c.close()


def _alpha_series(n_runs, n_steps, seed, symmetric=False):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_runs):
        a = np.cumsum(rng.normal(size=(n_steps, 3, 3)), axis=0) * 0.05 + rng.normal(size=(1, 3, 3))
        t = np.arange(n_steps)[:, None, None]
        a = a + 0.3 * np.cos(0.21 * t) * rng.normal(size=(1, 3, 3))
        if symmetric:
            a = 0.5 * (a + a.transpose(0, 2, 1))
        out.append(a.reshape(n_steps, 9))
    return np.array(out)


def _orientations(rng, n):
    nh = rng.normal(size=(n, 3))
    eh = rng.normal(size=(n, 3))
    nh /= np.linalg.norm(nh, axis=1, keepdims=True)
    eh /= np.linalg.norm(eh, axis=1, keepdims=True)
    nh[:2] = [[1, 0, 0], [1, 0, 0]]  # Z(XX)Z-bar and Z(XY)Z-bar
    eh[:2] = [[1, 0, 0], [0, 1, 0]]
    return nh, eh


@pytest.mark.parametrize("window,flags,laser", [(0, 0, 0.0), (1, 1, 0.0), (0, 1, 15000.0)])
def test_raman_map(gpu_lib, ctx, window, flags, laser):
    series = _alpha_series(2, 600, 11)
    nh, eh = _orientations(np.random.default_rng(12), 7)
    f, S = gpu_lib.tnep_raman_map(ctx, series, 2.0, 200, nh, eh, window=window, flags=flags, laser_cm1=laser)
    fr, Sr = oracle.raman_map(list(series), 2.0, 200, nh, eh, window=(window == 0), subtract_mean=bool(flags & 1),
                              laser_cm1=laser if laser > 0 else None)
    assert np.allclose(f, fr, rtol=1e-14, atol=0)
    err = max(spectrum_error(S[o], Sr[o]) for o in range(len(nh)))
    print("map error", err, flush=True)
    assert err <= SPECTRUM_TOL


def test_raman_map_device_series(gpu_lib, ctx):
    import torch

    series = _alpha_series(1, 300, 13)
    nh, eh = _orientations(np.random.default_rng(14), 3)
    f, S = gpu_lib.tnep_raman_map(ctx, series, 1.0, 100, nh, eh)
    ds = torch.as_tensor(series).cuda()
    df = torch.zeros(101, dtype=torch.float64, device="cuda")
    dS = torch.zeros((3, 101), dtype=torch.float64, device="cuda")
    gpu_lib.tnep_raman_map(ctx, ds, 1.0, 100, nh, eh, freq=df, intensity=dS)
    torch.cuda.synchronize()
    assert np.array_equal(dS.cpu().numpy(), S) and np.array_equal(df.cpu().numpy(), f)


@pytest.mark.parametrize("kind", [1, 2, 3])
def test_laser_prefactor(gpu_lib, ctx, kind):
    series = _alpha_series(2, 400, 15)
    nh, eh = (0.6, 0.8, 0.0), (0.0, 0.0, 1.0)
    _, S, _ = gpu_lib.tnep_spectrum(ctx, series, kind, 1.0, 150, n_hat=nh, e_hat=eh, laser_cm1=20000.0)
    _, Sr, _ = oracle.spectrum(list(series), kind, 1.0, 150, n_hat=nh, e_hat=eh, laser_cm1=20000.0)
    assert spectrum_error(S, Sr) <= SPECTRUM_TOL


def _chunks(n, rng):
    sizes = []
    while sum(sizes) < n:
        sizes.append(int(rng.choice([1, 7, 64, 311, 1000])))
    sizes[-1] -= sum(sizes) - n
    return [s for s in sizes if s > 0]


@pytest.mark.parametrize("kind", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("flags", [0, 1])
def test_stream_matches_whole_runs(gpu_lib, ctx, kind, flags):
    """Two runs of different lengths pushed in irregular chunks (single
    samples included) equal the oracle on the whole runs."""
    rng = np.random.default_rng(20 + kind)
    runs = [_alpha_series(1, n, 30 + n)[0] for n in (900, 700)]
    if kind == 0:
        runs = [r[:, :3] for r in runs]
    nh, eh = (0.0, 0.6, 0.8), (1.0, 0.0, 0.0)
    st = gpu_lib.AcfStream(ctx, kind, 120, flags=flags, n_hat=nh, e_hat=eh)
    for r in runs:
        pos = 0
        for sz in _chunks(len(r), rng):
            st.push(r[pos:pos + sz])
            pos += sz
        st.end_run()
    if kind == 4:
        onh, oeh = _orientations(rng, 4)
        f, S = st.raman_map(1.0, onh, oeh)
        _, Sr = oracle.raman_map(runs, 1.0, 120, onh, oeh, subtract_mean=bool(flags))
        err = max(spectrum_error(S[o], Sr[o]) for o in range(4))
    else:
        f, S, a = st.spectrum(1.0)
        _, Sr, Cr = oracle.spectrum(runs, kind, 1.0, 120, n_hat=nh, e_hat=eh, subtract_mean=bool(flags))
        err = spectrum_error(S, Sr)
        assert np.abs(a - Cr).max() <= 1e-9 * np.abs(Cr).max()
    st.close()
    print(f"stream kind {kind} flags {flags}: {err:.2e}", flush=True)
    assert err <= SPECTRUM_TOL


def test_stream_long_runs_and_device_chunks(gpu_lib, ctx):
    """10^5-sample runs (the paper's trajectories are 10^5-2x10^5 samples),
    pushed as device tensors in 8192-sample chunks."""
    import torch

    rng = np.random.default_rng(40)
    runs = [_alpha_series(1, 100000, 41 + k, symmetric=True)[0] for k in range(2)]
    st = gpu_lib.AcfStream(ctx, 2, 500)
    for r in runs:
        d = torch.as_tensor(r).cuda()
        for pos in range(0, len(r), 8192):
            st.push(d[pos:pos + 8192])
        st.end_run()
    f, S, _ = st.spectrum(5.0)
    st.close()
    _, Sr, _ = oracle.spectrum(runs, 2, 5.0, 500)
    err = spectrum_error(S, Sr)
    print("long stream error", err, flush=True)
    assert err <= SPECTRUM_TOL
    assert rng is not None


def test_stream_blocks_and_long_lags(gpu_lib, ctx):
    """Max lags up to 2048 split each chunk into blocks of 4096 - (M - 1) new
    samples, 32 blocks per launch round: one 70,000-sample push at M = 2048
    takes two rounds (35 blocks).  Longer lags (M = 2500) take one padded
    transform per chunk.  Both against the oracle's direct lag sums."""
    rng = np.random.default_rng(50)
    for M, sizes in ((2048, [70000, 3, 5000]), (2500, [1, 4000, 999, 3000])):
        runs = [_alpha_series(1, sum(sizes), 51 + M)[0], _alpha_series(1, 2 * M + 7, 52 + M)[0]]
        st = gpu_lib.AcfStream(ctx, 1, M, flags=1)
        for r, chunks in zip(runs, (sizes, [len(runs[1])])):
            pos = 0
            for sz in chunks:
                st.push(r[pos:pos + sz])
                pos += sz
            st.end_run()
        _, S, a = st.spectrum(2.0)
        st.close()
        _, Sr, Cr = oracle.spectrum(runs, 1, 2.0, M, subtract_mean=True)
        err = spectrum_error(S, Sr)
        acf_err = np.abs(a - Cr).max() / np.abs(Cr).max()
        print(f"max lag {M}: spectrum {err:.2e} acf {acf_err:.2e}", flush=True)
        assert acf_err <= 1e-9
        assert err <= SPECTRUM_TOL
    assert rng is not None


def test_stream_errors(gpu_lib, ctx):
    st = gpu_lib.AcfStream(ctx, 1, 50)
    st.push(np.zeros((20, 9)))
    with pytest.raises(gpu_lib.TnepError):
        st.end_run()  # shorter than max_lag
    with pytest.raises(gpu_lib.TnepError):
        st.spectrum(1.0)  # no finished run
    with pytest.raises(gpu_lib.TnepError):
        st.raman_map(1.0, [[1, 0, 0]], [[1, 0, 0]])  # not a map stream
    st.close()
    with pytest.raises(gpu_lib.TnepError):
        gpu_lib.AcfStream(ctx, 7, 50)
