"""tnep_spectrum_noalloc (the spectrum entry point that allocates nothing and
keeps its workspace in the library's fixed per-GPU array) against
tnep_spectrum on the same device inputs: two calls in a row, the second on a
smaller input (the array keeps the first call's contents), every spectrum
kind; the results must equal those of tnep_spectrum (same kernels) and meet
the spectrum bound against the oracle.  Oversized and host inputs are
rejected with an error."""
import numpy as np
import pytest
import torch

import oracle
from parity import SPECTRUM_TOL, spectrum_error

pytestmark = pytest.mark.gpu


def _series(n_series, n_steps, comps, seed):
    rng = np.random.default_rng(seed)
    t = np.arange(n_steps)[None, :, None]
    w = rng.uniform(0.05, 0.4, (n_series, 1, comps))
    return np.cos(w * t) + 0.3 * rng.standard_normal((n_series, n_steps, comps))


@pytest.mark.parametrize("kind,comps", [(0, 3), (1, 9), (2, 9), (3, 9)])
def test_noalloc_matches_allocating_call(gpu_lib, kind, comps):
    ctx = gpu_lib.Context(0)
    nh, eh = (0.0, 0.6, 0.8), (1.0, 0.0, 0.0)
    for n_series, n_steps, M, seed in ((3, 2500, 700, 1), (2, 900, 300, 2)):
        s = _series(n_series, n_steps, comps, seed + 10 * kind)
        d = torch.as_tensor(s).cuda()
        f_a = torch.zeros(M + 1, dtype=torch.float64, device="cuda")
        S_a = torch.zeros_like(f_a)
        C_a = torch.zeros(M, dtype=torch.float64, device="cuda")
        f_n = torch.full((M + 1,), float("nan"), dtype=torch.float64, device="cuda")
        S_n = torch.full_like(f_n, float("nan"))
        C_n = torch.full((M,), float("nan"), dtype=torch.float64, device="cuda")
        gpu_lib.tnep_spectrum(ctx, d, kind, 0.5, M, n_hat=nh, e_hat=eh, freq=f_a, intensity=S_a, acf=C_a)
        gpu_lib.tnep_spectrum_noalloc(ctx, d, kind, 0.5, M, f_n, S_n, C_n, n_hat=nh, e_hat=eh)
        torch.cuda.synchronize()
        assert torch.equal(f_n, f_a) and torch.equal(S_n, S_a) and torch.equal(C_n, C_a), (kind, n_steps)
        _, Sr, Cr = oracle.spectrum(list(s), kind, 0.5, M, n_hat=nh, e_hat=eh)
        err = spectrum_error(S_n.cpu().numpy(), Sr)
        print(f"kind {kind} n_steps {n_steps}: error vs oracle {err:.2e}", flush=True)
        assert err < SPECTRUM_TOL
        assert spectrum_error(C_n.cpu().numpy(), Cr) < 1e-10
    ctx.close()


def test_noalloc_rejects_what_it_cannot_hold(gpu_lib):
    ctx = gpu_lib.Context(0)
    M = 100
    f = torch.zeros(M + 1, dtype=torch.float64, device="cuda")
    S = torch.zeros_like(f)
    # 9 anisotropic signals x 64 runs x FFT length 2^14: 302 MB of workspace
    big = torch.zeros((64, 5000, 9), dtype=torch.float64, device="cuda")
    with pytest.raises(gpu_lib.TnepError) as e:
        gpu_lib.tnep_spectrum_noalloc(ctx, big, 2, 1.0, M, f, S)
    assert e.value.code == -6
    host = np.zeros((1, 500, 3))
    with pytest.raises(gpu_lib.TnepError) as e:
        gpu_lib.tnep_spectrum_noalloc(ctx, host, 0, 1.0, M, f, S)
    assert e.value.code == -1
    # a normal call after the rejected ones
    s = _series(1, 800, 3, 5)
    d = torch.as_tensor(s).cuda()
    gpu_lib.tnep_spectrum_noalloc(ctx, d, 0, 1.0, M, f, S)
    fa, Sa, _ = gpu_lib.tnep_spectrum(ctx, s, 0, 1.0, M)
    torch.cuda.synchronize()
    assert np.array_equal(S.cpu().numpy(), Sa)
    ctx.close()
