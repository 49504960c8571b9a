"""GPU parity: every entry point of libscint (through the C ABI binding)
against the FP64 oracle on the same seeded inputs.

Sizes span one to many workgroups, rows and transpose tiles, including ragged
tiles (N = 40, 100, 1000 are not multiples of the 64-wide transpose tile)
and the single-stage FFT (N = 16).

Tolerances: FP64 kernels agree with the oracle to rounding (max relative
1e-10); FP32 intensities meet the stated bar, RMS error <= 2e-5 and max error
<= 1e-3 of the mean intensity (the per-pixel relative error is undefined at
dark speckles); FP32 screens and gradients to a few 1e-6 of their RMS.
"""
import numpy as np
import pytest
import torch

import inputs

pytestmark = pytest.mark.gpu

F32_RMS, F32_MAX = 2e-5, 1e-3


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1301_0514_amd import scint
    scint.load_library()
    return scint


def dev(a, dtype):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    return t.detach().double().cpu().numpy()


def intensity_errors(I, I_ref):
    m = I_ref.mean()
    d = I - I_ref
    return np.sqrt(np.mean(d * d)) / m, np.abs(d).max() / m


def check_intensity(I, I_ref, dtype):
    e_rms, e_max = intensity_errors(I, I_ref)
    if dtype == torch.float64:
        assert e_max < 1e-10, (e_rms, e_max)
    else:
        assert e_rms < F32_RMS and e_max < F32_MAX, (e_rms, e_max)
    return e_rms, e_max


def check_field(x, x_ref, dtype, rms_tol=3e-6):
    scale = np.sqrt(np.mean(x_ref * x_ref))
    d = x - x_ref
    if dtype == torch.float64:
        assert np.abs(d).max() < 1e-10 * np.abs(x_ref).max()
    else:
        assert np.sqrt(np.mean(d * d)) < rms_tol * scale
        assert np.abs(d).max() < 30 * rms_tol * np.abs(x_ref).max()


DTYPES = [torch.float64, torch.float32]
SIZES = [16, 40, 64, 100, 256, 1000, 1024]


# ------------------------------------------------------------------ screen
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("N,R,beta", [(16, 2.0, 11 / 3), (40, 3.0, 3.2), (64, 4.0, 11 / 3), (100, 5.0, 3.9),
                                      (256, 4.0, 11 / 3), (1000, 8.0, 3.1), (2048, 24.0, 11 / 3)])
def test_screen(S, oracle, dtype, N, R, beta):
    # FP32 screens carry the lowest modes (|kx'|, |ky'| <= 16) in FP64 and
    # the rest through the FP32 transforms, so the stored screen is within a
    # few rounding units of FP32 of the exact one
    seed, r0, n = 17, 3, 2
    phi = host(S.ps_generate(N, 1.0, R, beta, seed, r0, n, dtype))
    for b in range(n):
        ref = oracle.screen(N, R, beta, seed, r0 + b)
        check_field(phi[b], ref, dtype, rms_tol=2e-7)


def test_screen_seed_high_word(S, oracle):
    N, seed = 64, (7 << 32) | 5
    phi = host(S.ps_generate(N, 1.0, 3.0, 11 / 3, seed, 0, 1, torch.float64))
    check_field(phi[0], oracle.screen(N, 3.0, 11 / 3, seed, 0), torch.float64)


def test_screen_physical_units(S, oracle):
    # R_diff and delta in any one unit: only R_diff/delta matters
    N = 64
    a = host(S.ps_generate(N, 28.85, 500.0, 11 / 3, 3, 0, 1, torch.float64))
    b = oracle.screen(N, 500.0 / 28.85, 11 / 3, 3, 0)
    check_field(a[0], b, torch.float64)


# ------------------------------------------------------------------ propagation
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("N", SIZES)
def test_propagate(S, oracle, dtype, N):
    rho = max(1.5, N / 16.0)
    s = 0.8
    phi = inputs.smooth_phase_field(N, seed=N, sigma=5.0, corr=2.0, n=2)
    phi = phi.astype(np.float32).astype(np.float64) if dtype == torch.float32 else phi
    lam = 5e-7
    z = 2 * np.pi * rho ** 2 / lam
    I = host(S.fresnel_propagate(dev(phi, dtype), 1.0, lam, z, s))
    for b in range(2):
        check_intensity(I[b], oracle.propagate(phi[b], rho, s), dtype)


@pytest.mark.parametrize("dtype", DTYPES)
def test_propagate_conjugate_plane_direct_sum(S, oracle, dtype):
    # N = 2 pi rho^2: equals the direct Fresnel sum of Eq. hxy (oracle-pinned)
    N = 16
    rho = np.sqrt(N / (2 * np.pi))
    phi = inputs.phase_field(N, seed=4, sigma=2.0)
    lam = 1e-6
    I = host(S.fresnel_propagate(dev(phi, dtype), 1.0, lam, 2 * np.pi * rho ** 2 / lam))
    check_intensity(I[0], oracle.fresnel_direct(phi[0], rho), dtype)


@pytest.mark.parametrize("dtype", DTYPES)
def test_uniform_screen_is_flat(S, dtype):
    N = 256
    phi = torch.full((1, N, N), 2.5, dtype=dtype, device="cuda")
    I = host(S.fresnel_propagate(phi, 1.0, 5e-7, 1e5))
    tol = 1e-12 if dtype == torch.float64 else 2e-6
    assert np.abs(I - 1).max() < tol


# ------------------------------------------------------------------ fused
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("N,R,rho", [(40, 2.5, 4.0), (256, 4.0, 32.0), (256, 4.0, 8.0), (1024, 8.0, 64.0)])
def test_screen_fresnel(S, oracle, dtype, N, R, rho):
    lam = 5e-7
    z = 2 * np.pi * rho ** 2 / lam
    I, phi = S.ps_screen_fresnel(N, 1.0, R, 11 / 3, 1, lam, z, first_realisation=0, n_real=2, dtype=dtype,
                                 want_phi=True)
    I, phi = host(I), host(phi)
    for b in range(2):
        ref_phi = oracle.screen(N, R, 11 / 3, 1, b)
        check_field(phi[b], ref_phi, dtype)
        check_intensity(I[b], oracle.propagate(ref_phi, rho), dtype)
    # the fused screen equals ps_generate's up to the rounding of two
    # differently scheduled kernels
    phi2 = host(S.ps_generate(N, 1.0, R, 11 / 3, 1, 0, 2, dtype))
    ulp = np.finfo(np.float64 if dtype == torch.float64 else np.float32).eps
    assert np.abs(phi - phi2).max() <= 8 * ulp * np.abs(phi).max()
    # without the screen returned the screens are made transposed and the
    # two propagation passes run in the other order (no final transpose):
    # the same pattern against the oracle
    I3 = host(S.ps_screen_fresnel(N, 1.0, R, 11 / 3, 1, lam, z, first_realisation=0, n_real=2, dtype=dtype))
    for b in range(2):
        check_intensity(I3[b], oracle.propagate(oracle.screen(N, R, 11 / 3, 1, b), rho), dtype)


# ------------------------------------------------------------------ polychromatic
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("N,n_lambda", [(64, 5), (100, 3), (256, 7), (40, 70)])
def test_polychromatic(S, oracle, dtype, N, n_lambda):
    lam_ref = 650e-9
    rho_ref = N / 10.0
    z = 2 * np.pi * rho_ref ** 2 / lam_ref
    lams = np.linspace(400e-9, 900e-9, n_lambda)
    w = np.random.default_rng(n_lambda).uniform(0.5, 2.0, n_lambda)
    phi = oracle.screen(N, 3.0, 11 / 3, 2, 0)[None]
    phi = np.concatenate([phi, oracle.screen(N, 3.0, 11 / 3, 2, 1)[None]])
    if dtype == torch.float32:
        phi = phi.astype(np.float32).astype(np.float64)
    I = host(S.illumination_polychromatic(dev(phi, dtype), 1.0, z, lam_ref, lams, w))
    for b in range(2):
        check_intensity(I[b], oracle.polychromatic(phi[b], 1.0, z, lam_ref, lams, w), dtype)


def test_polychromatic_equal_weights_default(S, oracle):
    N, lam_ref = 64, 6e-7
    z = 2 * np.pi * 6.0 ** 2 / lam_ref
    lams = [5e-7, 6e-7, 7e-7]
    phi = oracle.screen(N, 2.0, 11 / 3, 9, 0)[None]
    I = host(S.illumination_polychromatic(dev(phi, torch.float64), 1.0, z, lam_ref, lams))
    check_intensity(I[0], oracle.polychromatic(phi[0], 1.0, z, lam_ref, lams), torch.float64)


# ------------------------------------------------------------------ smear
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("N", [16, 40, 100, 256])
def test_smear(S, oracle, dtype, N):
    radii = [0.0, 0.5, 2.5, N / 6.0]
    I = inputs.intensity_field(N, seed=N, n=2)
    if dtype == torch.float32:
        I = I.astype(np.float32).astype(np.float64)
    out = host(S.source_smear(dev(I, dtype), 1.0, radii))
    assert out.shape == (2, len(radii), N, N)
    for b in range(2):
        for j, Rs in enumerate(radii):
            ref = oracle.smear(I[b], Rs)
            tol = 1e-11 if dtype == torch.float64 else 2e-6
            assert np.abs(out[b, j] - ref).max() < tol * np.abs(I[b]).max()


@pytest.mark.parametrize("n", [3, 5])
def test_smear_pairs_and_odd_batch(S, oracle, n):
    # realisations share complex transforms two by two; the odd last one
    # goes alone -- every output against the oracle, several radii
    N = 100
    radii = [0.0, 3.0, 11.0]
    I = inputs.intensity_field(N, seed=40 + n, n=n)
    out = host(S.source_smear(dev(I, torch.float64), 1.0, radii))
    assert out.shape == (n, len(radii), N, N)
    for b in range(n):
        for j, Rs in enumerate(radii):
            assert np.abs(out[b, j] - oracle.smear(I[b], Rs)).max() < 1e-11 * np.abs(I[b]).max()
    # in place with one radius
    t = dev(I, torch.float64)
    S.source_smear(t, 1.0, [3.0], out=t.view(n, 1, N, N))
    for b in range(n):
        assert np.abs(host(t)[b] - oracle.smear(I[b], 3.0)).max() < 1e-11 * np.abs(I[b]).max()


def test_smear_in_place_and_units(S, oracle):
    N = 64
    I = inputs.intensity_field(N, seed=3)
    t = dev(I, torch.float64)
    S.source_smear(t, 2.0, [7.0], out=t.view(1, 1, N, N))
    # radius 7 in units where delta = 2 is 3.5 pixels
    assert np.abs(host(t)[0] - oracle.smear(I[0], 3.5)).max() < 1e-11


# ------------------------------------------------------------------ adjoint
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("N,rho,s", [(40, 3.0, 1.0), (64, 5.0, 0.7), (256, 6.0, 1.0), (1000, 20.0, 1.2)])
def test_vjp(S, oracle, dtype, N, rho, s):
    phi = inputs.smooth_phase_field(N, seed=5, sigma=4.0, corr=2.0, n=2)
    gI = inputs.phase_field(N, seed=6, sigma=1.0, n=2)
    if dtype == torch.float32:
        phi = phi.astype(np.float32).astype(np.float64)
        gI = gI.astype(np.float32).astype(np.float64)
    lam = 5e-7
    z = 2 * np.pi * rho ** 2 / lam
    phi_d = dev(phi, dtype)
    # recomputing the forward field, and from the forward's checkpoint
    g, dots = S.fresnel_propagate_vjp(phi_d, 1.0, lam, z, dev(gI, dtype), s, want_dot=True)
    I_f, field = S.fresnel_propagate_field(phi_d, 1.0, lam, z, s)
    g_c, dots_c = S.fresnel_propagate_vjp(phi_d, 1.0, lam, z, dev(gI, dtype), s, want_dot=True, field=field)
    g, g_c, I_f, field = host(g), host(g_c), host(I_f), host(field)
    for b in range(2):
        ref = oracle.propagate_vjp(phi[b], rho, s, gI[b])
        tol = 1e-9 if dtype == torch.float64 else 1e-4
        ref_dot = (phi[b] * ref).sum()
        for gg, dd in ((g[b], dots[b]), (g_c[b], dots_c[b])):
            check_field(gg, ref, dtype, rms_tol=2e-5)
            assert abs(dd - ref_dot) <= tol * (np.abs(phi[b] * ref).sum())
        # the checkpoint is the field A, [x][y], with |A|^2 the pattern
        I_ref, A_ref = oracle.propagate(phi[b], rho, s, return_field=True)
        A = field[b, ..., 0] + 1j * field[b, ..., 1]
        check_field(np.abs(A.T) ** 2, I_ref, dtype)
        assert np.abs(A.T - A_ref).max() < (1e-10 if dtype == torch.float64 else 1e-5) * np.abs(A_ref).max()
        check_field(I_f[b], I_ref, dtype)


def test_autograd_matches_vjp(S, oracle):
    N, rho = 64, 5.0
    lam = 5e-7
    z = 2 * np.pi * rho ** 2 / lam
    phi_np = inputs.smooth_phase_field(N, seed=8, sigma=3.0, n=1)
    It_np = inputs.intensity_field(N, seed=9)
    phi = dev(phi_np, torch.float64).requires_grad_(True)
    It = dev(It_np, torch.float64)
    I = S.fresnel_intensity(phi, 1.0, lam, z)
    loss = ((I - It) ** 2).sum()
    loss.backward()
    ref = oracle.propagate_vjp(phi_np[0], rho, 1.0, 2 * (oracle.propagate(phi_np[0], rho) - It_np[0]))
    assert np.abs(host(phi.grad)[0] - ref).max() < 1e-9 * np.abs(ref).max()


# ------------------------------------------------------------------ reductions
@pytest.mark.parametrize("dtype", DTYPES)
def test_modulation_index_and_loss(S, oracle, dtype):
    N = 100
    I = inputs.intensity_field(N, seed=1, n=3) + 0.25
    It = inputs.intensity_field(N, seed=2, n=3)
    if dtype == torch.float32:
        I = I.astype(np.float32).astype(np.float64)
        It = It.astype(np.float32).astype(np.float64)
    m, mean = S.ps_modulation_index(dev(I, dtype), want_mean=True)
    for b in range(3):
        assert m[b] == pytest.approx(oracle.modulation_index(I[b]), rel=1e-12)
        assert mean[b] == pytest.approx(I[b].mean(), rel=1e-13)
    loss, grad = S.ps_l2_loss(dev(I, dtype), dev(It, dtype))
    for b in range(3):
        assert loss[b] == pytest.approx(((I[b] - It[b]) ** 2).sum(), rel=1e-6 if dtype == torch.float32 else 1e-12)
    assert np.abs(host(grad) - 2 * (I - It)).max() < (1e-6 if dtype == torch.float32 else 1e-13) * 10


# ------------------------------------------------------------------ determinism
def test_bitwise_reproducible(S):
    N = 1024
    a = S.ps_screen_fresnel(N, 1.0, 8.0, 11 / 3, 1, 5e-7, 2 * np.pi * 64 ** 2 / 5e-7)
    b = S.ps_screen_fresnel(N, 1.0, 8.0, 11 / 3, 1, 5e-7, 2 * np.pi * 64 ** 2 / 5e-7)
    assert torch.equal(a, b)
    m1 = S.ps_modulation_index(a)
    m2 = S.ps_modulation_index(b)
    assert m1 == m2


# ------------------------------------------------------------------ graph capture
def test_graph_replay_matches_eager(S):
    """The batched step captured into a HIP graph: every replay, with eager
    work and synchronisations between replays, equals the eager result."""
    N, n_real = 256, 2
    lams = np.linspace(450e-9, 850e-9, 5)
    z = 2 * np.pi * 20.0 ** 2 / 650e-9
    radii = [3.0, 9.0]
    phi = torch.empty((n_real, N, N), dtype=torch.float32, device="cuda")
    I = torch.empty_like(phi)
    ext = torch.empty((n_real, len(radii), N, N), dtype=torch.float32, device="cuda")

    def step():
        S.ps_generate(N, 1.0, 4.0, 11 / 3, 5, 0, n_real, out=phi)
        S.illumination_polychromatic(phi, 1.0, z, 650e-9, lams, out=I)
        S.source_smear(I, 1.0, radii, out=ext)

    g, stream = S.capture_graph(step, warmup=2)
    with torch.cuda.stream(stream):
        step()
    stream.synchronize()
    ref_I, ref_ext = I.clone(), ext.clone()
    for rep in range(3):
        I.fill_(-1.0)
        ext.fill_(-1.0)
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            g.replay()
        stream.synchronize()
        assert torch.equal(I, ref_I), rep
        assert torch.equal(ext, ref_ext), rep
        # eager work between replays
        S.ps_screen_fresnel(128, 1.0, 3.0, 11 / 3, 1, 5e-7, 1e4)
        torch.cuda.synchronize()


def test_cold_call_under_capture_returns_status(S, oracle):
    """A first call of a size (tables to build, workspace to allocate) made
    while its stream is being captured returns PS_E_CAPTURE and enqueues
    nothing; so do entry points that return host values.  After one call
    outside the capture, the same call captures and its replays equal the
    oracle's pattern."""
    N, rho = 320, 20.0
    z = 2 * np.pi * rho ** 2 / 5e-7
    phi = dev(inputs.smooth_phase_field(N, seed=3, sigma=2.0, corr=4.0), torch.float32)
    out = torch.empty_like(phi)
    S.release_cache()
    stream = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with pytest.raises(S.ScintError) as e:
        with torch.cuda.graph(g, stream=stream):
            out.zero_()
            S.fresnel_propagate(phi, 1.0, 5e-7, z, out=out)
    assert e.value.code == S.PS_E_CAPTURE
    g2 = torch.cuda.CUDAGraph()
    with pytest.raises(S.ScintError) as e:
        with torch.cuda.graph(g2, stream=stream):
            out.zero_()
            S.ps_modulation_index(phi)
    assert e.value.code == S.PS_E_CAPTURE
    # warm on the capture stream, then capture and replay
    S.tune_plans(N)
    with torch.cuda.stream(stream):
        S.fresnel_propagate(phi, 1.0, 5e-7, z, out=out)
    stream.synchronize()
    g3 = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g3, stream=stream):
        S.fresnel_propagate(phi, 1.0, 5e-7, z, out=out)
    I_ref = oracle.propagate(host(phi)[0], rho)
    for rep in range(2):
        out.fill_(-1.0)
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            g3.replay()
        stream.synchronize()
        d = host(out)[0] - I_ref
        assert np.sqrt(np.mean(d * d)) / I_ref.mean() < F32_RMS, rep
