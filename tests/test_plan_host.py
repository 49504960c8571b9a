"""Host planning of illumination_polychromatic (ps_plan_polychromatic): the
split into jobs and the workspace a call takes, computed without a GPU.

The rules: in FP32 from N = 2048 up the jobs are pipelined when four complex
buffers of one job's grids fit the budget and the work makes two or more jobs
(work that fits one job is split in two, by realisations, else wavelengths);
otherwise the plain loop takes chunks of up to 64 wavelengths whose two
complex buffers fit.  Sizes below follow the bench's configuration (8192^2,
8 realisations, 32 wavelengths), the paper's K_s run (20000^2, 21
wavelengths) and small budgets that force chunking.
"""
import pytest
import torch

GiB = 1 << 30
MiB = 1 << 20


@pytest.fixture(scope="module")
def S():
    from paper_1301_0514_amd import scint
    try:
        scint.load_library()
    except FileNotFoundError:
        pytest.skip("library not built")
    return scint


def pipelined_ws(N, C, nb):
    return 4 * 8 * N * N * C * nb + 4 * N * N * nb + 3 * C * N * 8 + 4096


def test_bench_configuration(S, monkeypatch):
    monkeypatch.delenv("SCINT_PIPELINE", raising=False)
    p = S.plan_polychromatic(8192, 8, 32, 96 * GiB)
    assert p == {"pipelined": True, "n_jobs": 8, "lambdas_per_job": 32, "real_per_job": 1,
                 "workspace_bytes": pipelined_ws(8192, 32, 1)}
    assert p["workspace_bytes"] <= 96 * GiB


def test_work_that_fits_one_job_is_split_in_two(S, monkeypatch):
    monkeypatch.delenv("SCINT_PIPELINE", raising=False)
    # by realisations ...
    p = S.plan_polychromatic(2048, 8, 32, 96 * GiB)
    assert (p["pipelined"], p["n_jobs"], p["real_per_job"], p["lambdas_per_job"]) == (True, 2, 4, 32)
    p = S.plan_polychromatic(2048, 5, 3, 96 * GiB)
    assert (p["n_jobs"], p["real_per_job"]) == (2, 3)
    # ... else by wavelengths
    p = S.plan_polychromatic(8192, 1, 32, 96 * GiB)
    assert (p["pipelined"], p["n_jobs"], p["real_per_job"], p["lambdas_per_job"]) == (True, 2, 1, 16)
    p = S.plan_polychromatic(8192, 1, 5, 96 * GiB)
    assert (p["n_jobs"], p["lambdas_per_job"]) == (2, 3)
    # one realisation and one wavelength cannot be split: the plain loop
    p = S.plan_polychromatic(8192, 1, 1, 96 * GiB)
    assert (p["pipelined"], p["n_jobs"]) == (False, 1)


def test_small_budget_halves_the_wavelengths_per_job(S, monkeypatch):
    monkeypatch.delenv("SCINT_PIPELINE", raising=False)
    p = S.plan_polychromatic(2048, 3, 8, 300 * MiB)
    assert p == {"pipelined": True, "n_jobs": 12, "lambdas_per_job": 2, "real_per_job": 1,
                 "workspace_bytes": pipelined_ws(2048, 2, 1)}
    assert p["workspace_bytes"] <= 300 * MiB
    # two realisations per job when they fit
    p = S.plan_polychromatic(2048, 5, 2, 600 * MiB)
    assert (p["n_jobs"], p["real_per_job"], p["lambdas_per_job"]) == (3, 2, 2)


def test_paper_ks_configuration(S, monkeypatch):
    monkeypatch.delenv("SCINT_PIPELINE", raising=False)
    p = S.plan_polychromatic(20000, 1, 21, 96 * GiB)
    assert (p["pipelined"], p["n_jobs"], p["lambdas_per_job"], p["real_per_job"]) == (True, 4, 6, 1)


def test_plain_loop_cases(S, monkeypatch):
    monkeypatch.delenv("SCINT_PIPELINE", raising=False)
    # a pipelined job does not fit (144 MiB) but a plain chunk does (80 MiB)
    p = S.plan_polychromatic(2048, 2, 1, 100 * MiB)
    assert (p["pipelined"], p["n_jobs"], p["lambdas_per_job"], p["real_per_job"]) == (False, 2, 1, 1)
    assert p["workspace_bytes"] <= 100 * MiB
    # below 2048 and in FP64 the plain loop
    assert not S.plan_polychromatic(1024, 8, 32, 96 * GiB)["pipelined"]
    # (FP64 4096^2 x 32 wavelengths: 2 x 16 GiB + 128 MiB per realisation, 5 per chunk)
    q = S.plan_polychromatic(4096, 8, 32, 96 * GiB, dtype=torch.float64)
    assert (q["pipelined"], q["n_jobs"], q["real_per_job"], q["lambdas_per_job"]) == (False, 2, 5, 32)
    # and when the environment turns the pipeline off
    monkeypatch.setenv("SCINT_PIPELINE", "0")
    p = S.plan_polychromatic(8192, 8, 32, 96 * GiB)
    assert (p["pipelined"], p["n_jobs"], p["real_per_job"]) == (False, 4, 2)


def test_plan_rejects_bad_arguments(S):
    with pytest.raises(S.ScintError):
        S.plan_polychromatic(1234, 1, 1, GiB)
    with pytest.raises(S.ScintError):
        S.plan_polychromatic(2048, 1, 5000, GiB)
    with pytest.raises(ValueError):
        S.plan_polychromatic(2048, 1, 1, 0)
