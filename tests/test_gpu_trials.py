"""GPU parity of plv_over_trials (Lachaux's PLV across trials, Eq. 1; matrix
form Eq. 8) against the FP64 oracle, element by element at every time point
of the window.  Trials are lagged-oscillator mixtures drawn independently, so
the zero-lag-mixed channel pairs (2m, 2m+1) stay locked across trials and the
others do not.  Tolerances are those of the other parity tests."""
import numpy as np
import pytest

import oracle
import synth
from tests.test_gpu_parity import TOL, compare

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def plv_mod():
    import paper_1710_08037_amd as plv
    return plv


def trials(ntr, n, t, seed):
    return np.stack([synth.glag_analytic(n, t, 1000.0, 4, (8, 12), seed=seed + k) for k in range(ntr)])


def to_dev(z, prec):
    dt = np.complex128 if prec == "f64" else np.complex64
    return torch.from_numpy(np.ascontiguousarray(z.astype(dt))).cuda()


def exact(z, prec):
    return z.astype(np.complex128 if prec == "f64" else np.complex64).astype(np.complex128)


def check(out, ref, prec, where):
    got = {k: v.cpu().numpy().astype(np.complex128 if k == "g" else np.float64) for k, v in out.items()}
    for t in range(ref["plv"].shape[0]):
        compare({k: got[k][t] for k in got}, {k: ref[k][t] for k in ref}, TOL[prec], "%s t=%d" % (where, t))


@pytest.mark.parametrize("prec", ["f64", "f32", "split_bf16", "bf16", "f16"])
def test_trial_major_against_oracle(prec):
    ntr, n, t = 40, 37, 30
    z = trials(ntr, n, t, seed=synth.seed_for(7))
    out = plv_mod().over_trials(to_dev(z, prec), prec=prec, want_g=True)
    torch.cuda.synchronize()
    check(out, oracle.full_over_trials(exact(z, prec)), prec, "trial-major %s" % prec)


@pytest.mark.parametrize("prec", ["f32", "split_bf16"])
def test_signals_samples_trials_view_and_window(prec):
    """Data stored signals x samples x trials (trials fastest), passed as a
    permuted view; a window of time points."""
    ntr, n, t = 24, 20, 50
    z = trials(ntr, n, t, seed=synth.seed_for(7, 5))
    stored = to_dev(np.transpose(z, (1, 2, 0)), prec)     # [n, t, ntr], contiguous
    view = stored.permute(2, 0, 1)                         # [ntr, n, t] view, strides (1, t*ntr, ntr)
    win = (7, 43)
    out = plv_mod().over_trials(view, prec=prec, window=win, want_g=True)
    torch.cuda.synchronize()
    check(out, oracle.full_over_trials(exact(z, prec), window=win), prec, "view %s" % prec)


@pytest.mark.parametrize("prec", ["f32", "split_bf16"])
def test_single_time_point_many_trials(prec):
    """One time point (a single Gram problem, K-chunked over 3000 trials)."""
    ntr, n, t = 3000, 48, 3
    z = trials(1, n, ntr, seed=synth.seed_for(7, 9))[0].T[:, :, None]   # [ntr, n, 1] from one long signal
    z = np.ascontiguousarray(np.repeat(z, t, axis=2))
    out = plv_mod().over_trials(to_dev(z, prec), prec=prec, window=(1, 2), want_g=True)
    torch.cuda.synchronize()
    check(out, oracle.full_over_trials(exact(z, prec), window=(1, 2)), prec, "single %s" % prec)


def test_many_time_points_sampled():
    """148 signals, 40 trials, 500 time points (500 grouped problems): every
    pair at 8 sampled time points."""
    ntr, n, t = 40, 148, 500
    z = trials(ntr, n, t, seed=synth.seed_for(7, 20)).astype(np.complex64)
    out = plv_mod().over_trials(to_dev(z, "split_bf16"), prec="split_bf16", want_g=True)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy().astype(np.complex128 if k == "g" else np.float64) for k, v in out.items()}
    for tt in np.random.default_rng(4).choice(t, size=8, replace=False):
        ref = oracle.full_over_trials(exact(z, "split_bf16"), window=(int(tt), int(tt) + 1))
        compare({k: got[k][tt] for k in got}, {k: ref[k][0] for k in ref}, TOL["split_bf16"], "t=%d" % tt)


@pytest.mark.parametrize("prec", ["f64", "f32", "split_bf16", "bf16", "f16"])
@pytest.mark.parametrize("n,ntr", [(192, 64), (150, 33), (64, 16), (1, 5), (192, 65), (193, 40), (70, 48), (100, 9)])
def test_small_problem_edges(prec, n, ntr):
    """Row and trial counts at tile and stage boundaries (192 rows = three
    64-wide tiles, 48 and 64 trials = three and four 16-sample stages) and
    just past them, every element of every matrix, G included and left out.
    The trials are padded only to the mode's K-unit (4, 8, 16 or 32), so
    most counts here end inside the last 32-trial block of the transpose."""
    t = 6
    z = trials(ntr, n, t, seed=synth.seed_for(7, 30 + n + ntr))
    for want_g in (True, False):
        out = plv_mod().over_trials(to_dev(z, prec), prec=prec, want_g=want_g)
        torch.cuda.synchronize()
        ref = oracle.full_over_trials(exact(z, prec))
        if want_g:
            check(out, ref, prec, "n=%d ntr=%d %s" % (n, ntr, prec))
        else:
            assert out["g"] is None
            got = {k: v.cpu().numpy().astype(np.float64) for k, v in out.items() if v is not None}
            for tt in range(t):
                for k in ("plv", "iplv"):
                    assert np.abs(got[k][tt] - ref[k][tt]).max() <= TOL[prec]
