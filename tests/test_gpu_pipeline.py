"""GPU parity of the pipelined polychromatic propagation (Sect. 3.2.4, Eq.
phiNl): from N = 2048 up in FP32, with two or more jobs, the transpose
between the x and y passes of one job runs as extra workgroups of the
neighbouring jobs' row passes.

The pipelined path must give the plain chunk loop's result bit for bit when
both split the work into the same jobs; the workspace budgets below are
chosen so that they do (comments give the job split).  Against the FP64
oracle the usual FP32 bar holds (RMS 2e-5, max 1e-3 of the mean).

Cases: many jobs of two wavelengths; a ragged last wavelength chunk; ragged
transpose units (N = 4000 is not a multiple of 128 or 64) with 200-thread
row workgroups, and 128-thread ones (4096, plan 0), where threads take two
lane roles of the transpose; the bench's shape (8192, 32 wavelengths, two realisations: two
jobs); the pipeline's prologue and epilogue with two and three jobs.  The
sections at the end check the same property for the source smear and the
screens, whose passes carry each other's transposes in the same way.
"""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

MiB = 1 << 20
F32_RMS, F32_MAX = 2e-5, 1e-3


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1301_0514_amd import scint
    scint.load_library()
    return scint


@pytest.fixture(scope="module")
def P():
    from paper_1301_0514_amd import presets
    return presets


def poly(S, monkeypatch, phi, z, lam_ref, lams, w, budget, pipeline):
    monkeypatch.setenv("SCINT_PIPELINE", "1" if pipeline else "0")
    S.set_workspace_budget(budget)
    try:
        out = S.illumination_polychromatic(phi, 1.0, z, lam_ref, lams, w)
        torch.cuda.synchronize()
        return out
    finally:
        S.set_workspace_budget(0)


def geometry(N, n_lambda, seed):
    lam_ref = 650e-9
    rho_ref = N / 12.0
    z = 2 * np.pi * rho_ref ** 2 / lam_ref
    lams = list(np.linspace(400e-9, 900e-9, n_lambda))
    w = list(np.random.default_rng(seed).uniform(0.5, 2.0, n_lambda))
    return z, lam_ref, lams, w


# (N, n_real, n_lambda, pipelined budget, plain budget): both give jobs of
#   2048: Cp = C = 2 wavelengths, one realisation (12 jobs; 6 jobs of 2, 2, 1)
#   2048 x 5 realisations: two wavelengths, two realisations (jobs of 2, 2, 1)
#   4000: one wavelength, one realisation (6 jobs)
#   4096: one wavelength, one realisation (4 jobs)
CASES = [(2048, 3, 8, 300 * MiB, 150 * MiB), (2048, 2, 5, 300 * MiB, 150 * MiB),
         (2048, 5, 2, 600 * MiB, 300 * MiB), (4000, 2, 3, 600 * MiB, 330 * MiB),
         (4096, 2, 2, 600 * MiB, 330 * MiB)]


@pytest.mark.parametrize("N,n_real,n_lambda,bp,bq", CASES)
def test_pipelined_equals_plain(S, monkeypatch, N, n_real, n_lambda, bp, bq):
    # the premise: the two budgets give the same split, pipelined and plain
    monkeypatch.setenv("SCINT_PIPELINE", "1")
    pl = S.plan_polychromatic(N, n_real, n_lambda, bp)
    monkeypatch.setenv("SCINT_PIPELINE", "0")
    ql = S.plan_polychromatic(N, n_real, n_lambda, bq)
    assert pl["pipelined"] and pl["n_jobs"] >= 2 and not ql["pipelined"]
    assert (pl["lambdas_per_job"], pl["real_per_job"]) == (ql["lambdas_per_job"], ql["real_per_job"])
    z, lam_ref, lams, w = geometry(N, n_lambda, N + n_lambda)
    if N == 4096:
        S.set_plan_variant(N, 0)  # the 128-thread plan
    try:
        phi = S.ps_generate(N, 1.0, N / 300.0, 11 / 3, 5, 0, n_real)
        a = poly(S, monkeypatch, phi, z, lam_ref, lams, w, bp, True)
        b = poly(S, monkeypatch, phi, z, lam_ref, lams, w, bq, False)
    finally:
        if N == 4096:
            S.set_plan_variant(N, -1)
    assert torch.equal(a, b)
    assert float(a.mean()) == pytest.approx(1.0, abs=1e-5)


@pytest.mark.parametrize("N,n_real,n_lambda,bp", [(2048, 2, 5, 300 * MiB), (4000, 1, 3, 600 * MiB)])
def test_pipelined_vs_oracle(S, oracle, monkeypatch, N, n_real, n_lambda, bp):
    z, lam_ref, lams, w = geometry(N, n_lambda, 3)
    phi = np.stack([oracle.screen(N, N / 300.0, 11 / 3, 8, r) for r in range(n_real)])
    phi32 = phi.astype(np.float32)
    I = poly(S, monkeypatch, torch.tensor(phi32, device="cuda"), z, lam_ref, lams, w, bp, True)
    I = I.double().cpu().numpy()
    for b in range(n_real):
        ref = oracle.polychromatic(phi32[b].astype(np.float64), 1.0, z, lam_ref, lams, w)
        m = ref.mean()
        d = I[b] - ref
        e_rms, e_max = np.sqrt(np.mean(d * d)) / m, np.abs(d).max() / m
        print("N=%d realisation %d e_rms=%.2e e_max=%.2e" % (N, b, e_rms, e_max))
        assert e_rms < F32_RMS and e_max < F32_MAX


@pytest.mark.parametrize("n_real", [2, 3])
def test_pipeline_prologue_and_epilogue(S, monkeypatch, n_real):
    # two jobs: the transpose of job 0 rides wholly on the x pass of job 1 and
    # that of job 1 wholly on the y pass of job 0; three jobs add one split
    N, n_lambda = 2048, 2
    z, lam_ref, lams, w = geometry(N, n_lambda, 1)
    phi = S.ps_generate(N, 1.0, 7.0, 11 / 3, 2, 0, n_real)
    a = poly(S, monkeypatch, phi, z, lam_ref, lams, w, 300 * MiB, True)   # jobs: one realisation, 2 wavelengths
    b = poly(S, monkeypatch, phi, z, lam_ref, lams, w, 150 * MiB, False)
    assert torch.equal(a, b)


@pytest.mark.parametrize("split,groups", [("0", None), ("1", None), ("0.3", "3:1:5:2"), (None, "1:1:1:1")])
def test_pipeline_split_settings(S, monkeypatch, split, groups):
    # every share and interleaving of the side transposes gives the same result
    N, n_real, n_lambda = 2048, 3, 4
    z, lam_ref, lams, w = geometry(N, n_lambda, 2)
    phi = S.ps_generate(N, 1.0, 7.0, 11 / 3, 4, 0, n_real)
    ref = poly(S, monkeypatch, phi, z, lam_ref, lams, w, 150 * MiB, False)
    if split is not None:
        monkeypatch.setenv("SCINT_SIDE_SPLIT", split)
    if groups is not None:
        monkeypatch.setenv("SCINT_SIDE_GROUPS", groups)
    a = poly(S, monkeypatch, phi, z, lam_ref, lams, w, 300 * MiB, True)
    assert torch.equal(a, ref)


def test_pipeline_bench_shape(S, P, monkeypatch):
    # the bench's polychromatic configuration with two realisations: the
    # pipelined path takes two jobs (64 GiB of workspace), the plain loop one
    c = P.POLY_8192
    N = c.N
    phi = S.ps_generate(N, 1.0, c.R_ref, c.beta, c.seed, 0, 2)
    GiB = 1 << 30
    a = poly(S, monkeypatch, phi, c.z, c.lam_ref, c.lambdas, None, 70 * GiB, True)   # jobs: one realisation each
    b = poly(S, monkeypatch, phi, c.z, c.lam_ref, c.lambdas, None, 70 * GiB, False)  # one job of both
    assert torch.equal(a, b)
    m = S.ps_modulation_index(a)
    assert all(0.05 < x < 1.5 for x in m)


def test_workspace_budget_rejects_tiny_values(S):
    with pytest.raises(S.ScintError):
        S.set_workspace_budget(1 << 20)
    with pytest.raises(ValueError):
        S.set_workspace_budget(-1)
    S.set_workspace_budget(0)


def test_pipeline_graph_replay_matches_eager(S):
    """The pipelined step (six jobs) captured into a HIP graph: every replay,
    with eager work and synchronisations between replays, equals the eager
    result bit for bit."""
    N, n_real, n_lambda = 2048, 3, 4
    z, lam_ref, lams, w = geometry(N, n_lambda, 6)
    radii = [5.0, 20.0]
    phi = torch.empty((n_real, N, N), dtype=torch.float32, device="cuda")
    I = torch.empty_like(phi)
    ext = torch.empty((n_real, len(radii), N, N), dtype=torch.float32, device="cuda")

    def step():
        S.ps_generate(N, 1.0, 7.0, 11 / 3, 9, 0, n_real, out=phi)
        S.illumination_polychromatic(phi, 1.0, z, lam_ref, lams, w, out=I)
        S.source_smear(I, 1.0, radii, out=ext)

    S.set_workspace_budget(300 * MiB)  # jobs: one realisation, two wavelengths
    try:
        g, stream = S.capture_graph(step, warmup=2)
        with torch.cuda.stream(stream):
            step()
        stream.synchronize()
    finally:
        S.set_workspace_budget(0)
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
        S.ps_screen_fresnel(128, 1.0, 3.0, 11 / 3, 1, 5e-7, 1e4)
        torch.cuda.synchronize()


def test_single_job_work_is_split_in_two(S, monkeypatch):
    # work that fits one job runs as two pipelined jobs: by realisations
    # (the same sums as the plain loop, so the same bits) ...
    N = 2048
    z, lam_ref, lams, w = geometry(N, 4, 7)
    phi = S.ps_generate(N, 1.0, 7.0, 11 / 3, 3, 0, 3)
    a = poly(S, monkeypatch, phi, z, lam_ref, lams, w, 0, True)
    b = poly(S, monkeypatch, phi, z, lam_ref, lams, w, 0, False)
    assert torch.equal(a, b)


def test_single_realisation_split_by_wavelength(S, oracle, monkeypatch):
    # ... or, for one realisation, by wavelengths (two partial sums: equal to
    # the plain loop to FP32 rounding, and within the bar of the oracle)
    N = 2048
    z, lam_ref, lams, w = geometry(N, 5, 8)
    phi = oracle.screen(N, 7.0, 11 / 3, 3, 0).astype(np.float32)
    phit = torch.tensor(phi[None], device="cuda")
    a = poly(S, monkeypatch, phit, z, lam_ref, lams, w, 0, True)
    b = poly(S, monkeypatch, phit, z, lam_ref, lams, w, 0, False)
    assert float((a - b).abs().max()) <= 4e-6 * float(b.abs().max())
    ref = oracle.polychromatic(phi.astype(np.float64), 1.0, z, lam_ref, lams, w)
    d = a[0].double().cpu().numpy() - ref
    m = ref.mean()
    assert np.sqrt(np.mean(d * d)) / m < F32_RMS and np.abs(d).max() / m < F32_MAX


@pytest.mark.parametrize("N,n", [(2048, 3), (4000, 2)])
def test_fresnel_propagate_pipelined_equals_plain(S, monkeypatch, N, n):
    # fresnel_propagate with several realisations takes the same pipeline
    # (one wavelength); its result is the plain loop's, bit for bit
    phi = S.ps_generate(N, 1.0, N / 300.0, 11 / 3, 6, 0, n)
    lam, s = 5e-7, 0.8
    z = 2 * np.pi * (N / 12.0) ** 2 / lam
    monkeypatch.setenv("SCINT_PIPELINE", "1")
    a = S.fresnel_propagate(phi, 1.0, lam, z, s)
    monkeypatch.setenv("SCINT_PIPELINE", "0")
    b = S.fresnel_propagate(phi, 1.0, lam, z, s)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("N", [10000, 16384])
def test_pipelined_equals_plain_large_workgroups(S, monkeypatch, N):
    # row workgroups of 1000 (10000, ragged transpose units) and 512 threads
    # (16384): threads beyond 256 only take part in the side transposes'
    # barriers.  A 48 GiB budget: two pipelined jobs of one realisation and
    # four wavelengths against one plain job of both, the same sums
    z, lam_ref, lams, w = geometry(N, 2, 4)
    budget = 48 << 30
    plan = S.plan_polychromatic(N, 2, 4, budget)
    assert plan["pipelined"] and plan["n_jobs"] == 2 and plan["lambdas_per_job"] == 4
    phi = S.ps_generate(N, 1.0, N / 300.0, 11 / 3, 12, 0, 2)
    a = poly(S, monkeypatch, phi, z, lam_ref, lams, w, budget, True)
    b = poly(S, monkeypatch, phi, z, lam_ref, lams, w, budget, False)
    assert torch.equal(a, b)
    assert float(a.mean()) == pytest.approx(1.0, abs=1e-5)


# ------------------------------------------------------------------ smear
# source_smear from N = 2048 up (FP32) with two or more realisation pairs runs
# its pairs as two jobs, each job's transposes carried by the other's passes;
# every pair's arithmetic is unchanged, so the result is the plain path's bit
# for bit.
@pytest.mark.parametrize("N,n_real,radii", [(2048, 4, [3.0]), (2048, 5, [2.0, 9.0, 30.0]),
                                            (2048, 8, [5.0, 20.0, 40.0, 80.0]), (4000, 4, [6.0, 25.0]),
                                            (10000, 4, [12.0])])
def test_smear_pipelined_equals_plain(S, monkeypatch, N, n_real, radii):
    g = torch.Generator(device="cuda").manual_seed(N + n_real)
    I = torch.rand((n_real, N, N), generator=g, device="cuda") + 0.5
    monkeypatch.setenv("SCINT_PIPELINE", "1")
    a = S.source_smear(I, 1.0, radii)
    monkeypatch.setenv("SCINT_PIPELINE", "0")
    b = S.source_smear(I, 1.0, radii)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_smear_pipelined_vs_oracle(S, oracle):
    import inputs
    N, radii = 2048, [4.0, 33.0]
    I = inputs.intensity_field(N, seed=21, n=4)
    out = S.source_smear(torch.tensor(I.astype(np.float32), device="cuda"), 1.0, radii)
    out = out.double().cpu().numpy()
    for b in (0, 3):
        for j, R in enumerate(radii):
            ref = oracle.smear(I[b].astype(np.float32).astype(np.float64), R)
            m = ref.mean()
            d = out[b, j] - ref
            assert np.sqrt(np.mean(d * d)) / m < F32_RMS and np.abs(d).max() / m < F32_MAX


# ------------------------------------------------------------------ screens
# ps_generate from N = 2048 up (FP32) splits a batch of realisations into up
# to four jobs; the noise pass of each job carries the transpose of the
# previous job's output and only the last job's transpose runs on its own.
# Every element is computed by the same code, so the screens equal the
# one-job path's bit for bit (SCINT_SCREEN_JOBS=1).
@pytest.mark.parametrize("N,n_real,jobs", [(2048, 8, "4"), (2048, 3, "4"), (2048, 5, "2"), (4000, 5, "4"),
                                           (10000, 2, "4"), (20000, 2, "4")])
def test_screen_pipelined_equals_plain(S, monkeypatch, N, n_real, jobs):
    monkeypatch.setenv("SCINT_SCREEN_JOBS", jobs)
    a = S.ps_generate(N, 1.0, N / 100.0, 11 / 3, 5, 7, n_real)
    monkeypatch.setenv("SCINT_SCREEN_JOBS", "1")
    b = S.ps_generate(N, 1.0, N / 100.0, 11 / 3, 5, 7, n_real)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("N,n_real,jobs", [(2048, 8, "4"), (4000, 5, "4")])
def test_transposed_screens_pipelined_equals_plain(S, monkeypatch, N, n_real, jobs):
    # ps_screen_fresnel without the screen returned makes its screens
    # transposed (noise along kx): the job split leaves every element's
    # arithmetic alike there too
    lam = 5e-7
    z = 2 * np.pi * (N / 20.0) ** 2 / lam
    monkeypatch.setenv("SCINT_SCREEN_JOBS", jobs)
    a = S.ps_screen_fresnel(N, 1.0, N / 100.0, 11 / 3, 5, lam, z, first_realisation=7, n_real=n_real)
    monkeypatch.setenv("SCINT_SCREEN_JOBS", "1")
    b = S.ps_screen_fresnel(N, 1.0, N / 100.0, 11 / 3, 5, lam, z, first_realisation=7, n_real=n_real)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_screen_pipelined_vs_oracle(S, oracle, monkeypatch):
    # eight realisations in four jobs: realisation 1 is transposed on the
    # second job's noise pass, realisation 7 by the last, standalone transpose
    monkeypatch.delenv("SCINT_SCREEN_JOBS", raising=False)
    N, R, seed, r0 = 2048, 24.0, 29, 40
    phi = S.ps_generate(N, 1.0, R, 11 / 3, seed, r0, 8).double().cpu().numpy()
    for b in (1, 7):
        ref = oracle.screen(N, R, 11 / 3, seed, r0 + b)
        d = phi[b] - ref
        scale = np.sqrt(np.mean(ref * ref))
        # the FP32 screen bar of the parity tests: RMS 3e-6, max 30 x that
        assert np.sqrt(np.mean(d * d)) < 3e-6 * scale
        assert np.abs(d).max() < 9e-5 * np.abs(ref).max()


# ------------------------------------------------------------------ x-pass split
# The pipelined x passes give each row two workgroups, each taking half of
# the job's wavelengths; the launcher keeps one where the row workgroups do
# not come in whole eights or a job has a single wavelength.  Every element
# is computed by the same code either way, so the result is unchanged bit
# for bit (SCINT_ITER_SPLIT=1 keeps one workgroup per row).
@pytest.mark.parametrize("N,n_real,n_lambda", [(2048, 2, 5), (2560, 2, 4), (4000, 1, 3), (8192, 1, 3)])
def test_x_pass_split_equals_unsplit(S, monkeypatch, N, n_real, n_lambda):
    z, lam_ref, lams, w = geometry(N, n_lambda, N)
    phi = S.ps_generate(N, 1.0, N / 100.0, 11 / 3, 3, 0, n_real)
    monkeypatch.setenv("SCINT_PIPELINE", "1")
    monkeypatch.setenv("SCINT_ITER_SPLIT", "2")
    a = S.illumination_polychromatic(phi, 1.0, z, lam_ref, lams, w)
    monkeypatch.setenv("SCINT_ITER_SPLIT", "1")
    b = S.illumination_polychromatic(phi, 1.0, z, lam_ref, lams, w)
    torch.cuda.synchronize()
    assert S.plan_polychromatic(N, n_real, n_lambda, 96 << 30)["pipelined"]
    assert torch.equal(a, b)


def test_screen_fresnel_pipelined_equals_plain(S, monkeypatch):
    # ps_screen_fresnel shares the screens' first pass and its job split
    N, n_real = 2048, 3
    rho = N / 12.0
    lam = 650e-9
    z = 2 * np.pi * rho ** 2 / lam
    monkeypatch.setenv("SCINT_SCREEN_JOBS", "4")
    Ia, pa = S.ps_screen_fresnel(N, 1.0, 20.0, 11 / 3, 9, lam, z, first_realisation=2, n_real=n_real, want_phi=True)
    monkeypatch.setenv("SCINT_SCREEN_JOBS", "1")
    Ib, pb = S.ps_screen_fresnel(N, 1.0, 20.0, 11 / 3, 9, lam, z, first_realisation=2, n_real=n_real, want_phi=True)
    torch.cuda.synchronize()
    assert torch.equal(pa, pb) and torch.equal(Ia, Ib)
