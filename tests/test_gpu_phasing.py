"""GPU phasing (section II-D: ER, HIO, shrinkwrap) against the FP64 oracle.

One step of each kind from the same float32 input is compared element by
element (float32 DFT contractions of length N per axis: 1e-5 relative to the
output norm is far above their rounding); where positivity decides a cell by
the sign of a rho' within the float32 error of zero, either branch is
accepted.  Twenty positivity-free HIO iterations stay within 1e-3 of the
oracle's trajectory; a full run from a random start recovers the object as
the oracle's does; shrinkwrap's blur matches to 1e-5 and its support
matches except at cells whose blur lies within float32 rounding of the
threshold.
"""
import ctypes

import numpy as np
import pytest
import torch

import paper_2109_05339_amd as spfel
from paper_2109_05339_amd import _lib
from oracle import phasing as ph
from tests._common import DEV, rel, gpu, host

pytestmark = pytest.mark.gpu


def blob_object(seed: int, N: int = 16):
    g = np.random.default_rng(seed)
    raw = np.zeros((N, N, N))
    a, b = N // 4, N // 4 + max(3, (7 * N) // 16)
    raw[a:b, a + 1:b + 1, a:b - 1] = g.random((b - a, b - a, b - a - 1))
    rho = ph.blur(raw, 0.7)
    sup = rho > 0.05 * rho.max()
    rho = np.where(sup, rho, 0.0)
    return rho, np.abs(np.fft.fftn(rho)), sup


def beam_stop(N, r=1.5):
    k = np.fft.fftfreq(N) * N
    K2 = k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2
    return K2 > r * r


def f32(x):
    return np.asarray(x, np.float32).astype(np.float64)


@pytest.mark.parametrize("N", [16, 17])
@pytest.mark.parametrize("mode", [spfel.PHASE_ER, spfel.PHASE_HIO])
@pytest.mark.parametrize("positivity", [False, True])
@pytest.mark.parametrize("masked", [False, True])
def test_one_step_against_oracle(N, mode, positivity, masked):
    rho, A, sup = blob_object(1, N)
    meas = beam_stop(N) if masked else None
    x = (np.random.default_rng(2).random((N, N, N)) * sup).astype(np.float32)
    A32 = A.astype(np.float32)
    p = spfel.Phase(N, device=DEV)
    r = gpu(x)
    err = p.iterate(r, gpu(A32), gpu(sup, torch.uint8), 1, mode=mode, beta=0.9,
                    positivity=positivity,
                    measured=None if meas is None else gpu(meas, torch.uint8), errors=True)
    got, e = host(r), float(host(err)[0])
    if mode == spfel.PHASE_ER:
        want, we = ph.er_step(f32(x), f32(A32), sup, meas, positivity)
    else:
        want, we = ph.hio_step(f32(x), f32(A32), sup, 0.9, meas, positivity)
    assert abs(e - we) <= 1e-5 * we
    rp, _ = ph.fourier_projection(f32(x), f32(A32), meas)
    close = np.abs(rp) <= 1e-5 * np.abs(rp).max()    # sign within float32 error of zero
    ok = ~(close & sup) if positivity else np.ones_like(sup)
    scale = np.linalg.norm(want)
    assert np.linalg.norm((got - want)[ok]) <= 1e-5 * scale
    if positivity:
        # the undecided cells took one of the two branches
        other = 0.0 if mode == spfel.PHASE_ER else f32(x) - 0.9 * rp
        amb = ~ok
        assert np.all(np.minimum(np.abs(got[amb] - rp[amb]), np.abs(got[amb] - np.broadcast_to(other, rp.shape)[amb]))
                      <= 1e-4 * np.abs(want).max())


def test_hio_trajectory_without_positivity():
    N = 16
    rho, A, sup = blob_object(3, N)
    x = (np.random.default_rng(4).random((N, N, N)) * sup).astype(np.float32)
    A32 = A.astype(np.float32)
    p = spfel.Phase(N, device=DEV)
    r = gpu(x)
    err = host(p.iterate(r, gpu(A32), gpu(sup, torch.uint8), 20, mode=spfel.PHASE_HIO, beta=0.9,
                         positivity=False, errors=True))
    want, errs = f32(x), []
    for _ in range(20):
        want, e = ph.hio_step(want, f32(A32), sup, 0.9, None, False)
        errs.append(e)
    assert rel(host(r), want) <= 1e-3
    assert rel(err, errs) <= 1e-3


def test_full_run_recovers_the_object():
    """300 HIO + 100 ER iterations with positivity from a random start in
    the true support: the error falls to float32 level and the density
    matches the object up to translation and inversion, as the oracle's run
    does."""
    N = 16
    rho, A, sup = blob_object(0, N)
    p = spfel.Phase(N, device=DEV)
    r = gpu((np.random.default_rng(10).random((N, N, N)) * sup).astype(np.float32))
    a, s = gpu(A.astype(np.float32)), gpu(sup, torch.uint8)
    p.iterate(r, a, s, 300, mode=spfel.PHASE_HIO, beta=0.9)
    err = host(p.iterate(r, a, s, 100, mode=spfel.PHASE_ER, errors=True))
    assert err[-1] < 1e-5
    assert np.all(err[1:] <= err[:-1] * (1 + 1e-3) + 1e-9)     # ER: non-increasing
    got = host(r).astype(np.float64)
    best = np.inf
    for cand in (got, np.roll(got[::-1, ::-1, ::-1], 1, axis=(0, 1, 2))):
        cc = np.fft.ifftn(np.fft.fftn(cand) * np.conj(np.fft.fftn(rho))).real
        sh = np.unravel_index(np.argmax(cc), cc.shape)
        al = np.roll(cand, [-sh[0], -sh[1], -sh[2]], axis=(0, 1, 2))
        best = min(best, np.linalg.norm(al - rho) / np.linalg.norm(rho))
    assert best < 5e-3


@pytest.mark.parametrize("N,sigma,tau", [(16, 1.0, 0.1), (17, 2.5, 0.2), (65, 1.5, 0.05)])
def test_shrinkwrap_against_oracle(N, sigma, tau):
    rho, _, _ = blob_object(5, N)
    x = (rho + 0.01 * np.random.default_rng(6).standard_normal(rho.shape)).astype(np.float32)
    p = spfel.Phase(N, device=DEV)
    s, b = p.shrinkwrap(gpu(x), sigma, tau, blurred=True)
    s, b = host(s).astype(bool), host(b)
    wb = ph.blur(np.abs(f32(x)), sigma)
    assert rel(b, wb) <= 1e-5
    ws = ph.shrinkwrap(f32(x), sigma, tau)
    near = np.abs(wb - tau * wb.max()) <= 1e-5 * wb.max()
    assert np.array_equal(s[~near], ws[~near])


def test_larger_grid_one_step():
    """N = 65 (the workload-2 model size): one HIO step with a beam stop."""
    N = 65
    rho, A, sup = blob_object(7, N)
    meas = beam_stop(N, 2.5)
    x = (np.random.default_rng(8).random((N, N, N)) * sup).astype(np.float32)
    p = spfel.Phase(N, device=DEV)
    r = gpu(x)
    p.iterate(r, gpu(A.astype(np.float32)), gpu(sup, torch.uint8), 1, mode=spfel.PHASE_HIO,
              positivity=False, measured=gpu(meas, torch.uint8))
    want, _ = ph.hio_step(f32(x), f32(A.astype(np.float32)), sup, 0.9, meas, False)
    assert rel(host(r), want) <= 1e-5


def test_argument_errors():
    p = spfel.Phase(8, device=DEV)
    z = torch.zeros((8, 8, 8), dtype=torch.float32, device=DEV)
    s = torch.ones((8, 8, 8), dtype=torch.uint8, device=DEV)
    L = spfel.lib()
    assert L.spfel_phase_iterate(p._h, z.data_ptr(), z.data_ptr(), None, s.data_ptr(), 1, 7, 0.9,
                                 1, None, None) == _lib.EINVAL
    assert L.spfel_phase_iterate(p._h, z.data_ptr(), z.data_ptr(), None, None, 1, 0, 0.9, 1,
                                 None, None) == _lib.EINVAL
    assert L.spfel_phase_shrinkwrap(p._h, z.data_ptr(), 0.0, 0.1, s.data_ptr(), None,
                                    None) == _lib.EINVAL
    assert L.spfel_phase_shrinkwrap(p._h, z.data_ptr(), 1.0, 1.5, s.data_ptr(), None,
                                    None) == _lib.EINVAL
    with pytest.raises(ValueError):
        p.iterate(torch.zeros((7, 7, 7), dtype=torch.float32, device=DEV), z, s, 1)
    torch.cuda.synchronize()
    p.close()
    assert L.spfel_phase_destroy(p._h) == _lib.ESTATE


def test_hio_step_at_the_workload_size():
    """N = 129, as the bench runs it: one HIO step with positivity off and a
    beam stop against the oracle over the whole grid."""
    N = 129
    g = np.random.default_rng(12)
    c = np.arange(N) - N // 2
    R2 = c[:, None, None] ** 2 + c[None, :, None] ** 2 + c[None, None, :] ** 2
    sup = R2 <= (N // 4) ** 2
    rho = g.random((N, N, N)) * sup
    A = np.abs(np.fft.fftn(rho)).astype(np.float32)
    x = (g.random((N, N, N)) * sup).astype(np.float32)
    meas = beam_stop(N, 3.0)
    p = spfel.Phase(N, device=DEV)
    r = gpu(x)
    err = p.iterate(r, gpu(A), gpu(sup, torch.uint8), 1, mode=spfel.PHASE_HIO, beta=0.9,
                    positivity=False, measured=gpu(meas, torch.uint8), errors=True)
    want, we = ph.hio_step(f32(x), f32(A), sup, 0.9, meas, False)
    assert rel(host(r), want) <= 1e-5
    assert abs(float(host(err)[0]) - we) <= 1e-5 * we


def test_zero_iterations_change_nothing():
    N = 8
    _, A, sup = blob_object(2, N)
    x = (np.random.default_rng(9).random((N, N, N)) * sup).astype(np.float32)
    p = spfel.Phase(N, device=DEV)
    r = gpu(x)
    err = p.iterate(r, gpu(A.astype(np.float32)), gpu(sup, torch.uint8), 0, errors=True)
    assert tuple(err.shape) == (0,)
    np.testing.assert_array_equal(host(r), x)
