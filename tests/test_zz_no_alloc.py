"""The entry point that allocates nothing, fresnel_propagate_noalloc, called
through the C ABI, against fresnel_propagate on the same inputs: two calls in
a row (the second smaller, so the shared scratch array holds the first
call's data when the second starts), in both precisions, and its refusal of
a batch that does not fit the array.

Tolerances: FP64 to rounding (1e-10 of the mean intensity); FP32 to the
intensity bar of the method (RMS <= 2e-5, max <= 1e-3 of the mean), since
the two entry points may use different FFT plans and twiddle roundings."""
import ctypes

import numpy as np
import pytest
import torch

import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1301_0514_amd import scint
    scint.load_library()
    return scint


def _call(S, phi, rho, s, out):
    lam = 5e-7
    z = 2 * np.pi * rho ** 2 / lam
    N = phi.shape[-1]
    n = phi.numel() // (N * N)
    lib = S.load_library()
    dt = S.PS_F64 if phi.dtype == torch.float64 else S.PS_F32
    rc = lib.fresnel_propagate_noalloc(N, 1.0, lam, z, S._ptr(phi), s, n, dt, S._ptr(out), S._stream(phi.device))
    return rc, S.fresnel_propagate(phi, 1.0, lam, z, phase_scale=s)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_noalloc_matches_fresnel_propagate(S, dtype):
    # (N, n screens, R_F px, phase scale); the second call is smaller
    cases = [(1024, 2, 40.0, 1.0), (256, 1, 12.0, 0.8)]
    for N, n, rho, s in cases:
        phi = torch.tensor(inputs.smooth_phase_field(N, seed=N + n, sigma=4.0, corr=3.0, n=n), dtype=dtype,
                           device="cuda")
        out = torch.full_like(phi, float("nan"))
        rc, ref = _call(S, phi, rho, s, out)
        torch.cuda.synchronize()
        assert rc == S.PS_OK, S.load_library().ps_last_error()
        I, I_ref = out.double().cpu().numpy(), ref.double().cpu().numpy()
        assert np.isfinite(I).all()
        m = I_ref.mean()
        e_rms = float(np.sqrt(np.mean((I - I_ref) ** 2)) / m)
        e_max = float(np.abs(I - I_ref).max() / m)
        print("noalloc %s N=%d n=%d: e_rms=%.2e e_max=%.2e" % (dtype, N, n, e_rms, e_max))
        if dtype == torch.float64:
            assert e_max < 1e-10
        else:
            assert e_rms < 2e-5 and e_max < 1e-3


def test_noalloc_rejects_batches_beyond_its_array(S):
    N, n = 2048, 2   # 2 x 2048^2 FP32 screens need 128 MiB of intermediates
    phi = torch.zeros((n, N, N), dtype=torch.float32, device="cuda")
    out = torch.full_like(phi, -1.0)
    lib = S.load_library()
    rc = lib.fresnel_propagate_noalloc(N, 1.0, 5e-7, 1e6, S._ptr(phi), 1.0, n, S.PS_F32, S._ptr(out),
                                       S._stream(phi.device))
    assert rc == -2
    assert b"scratch" in lib.ps_last_error()
    torch.cuda.synchronize()
    assert bool((out == -1.0).all())


def test_noalloc_captures_and_replays(S):
    """Captured into a HIP graph (what the entry point is for), every replay,
    with eager work and synchronisations between them, equals the eager call."""
    N, n, rho = 512, 2, 16.0
    lam = 5e-7
    z = 2 * np.pi * rho ** 2 / lam
    phi = torch.tensor(inputs.smooth_phase_field(N, seed=77, sigma=3.0, corr=3.0, n=n), dtype=torch.float32,
                       device="cuda")
    out = torch.empty_like(phi)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        S.fresnel_propagate_noalloc(phi, 1.0, lam, z, out=out)
    stream.synchronize()
    ref = out.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        S.fresnel_propagate_noalloc(phi, 1.0, lam, z, out=out)
    for rep in range(3):
        out.fill_(-1.0)
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            g.replay()
        stream.synchronize()
        assert torch.equal(out, ref), rep
        S.fresnel_propagate(phi[:1], 1.0, lam, z)  # eager work between replays
        torch.cuda.synchronize()
