"""Oracle pins for the overlaps Q, U, V of Eq. (QUV) computed from
frequency-domain inputs (the precompute before the likelihood): the
injection identity Q_m(t0) = sum_m' c_m' U_m,m' for data made of the modes
shifted to a grid time t0, Hermitian positive-semidefinite U and symmetric V,
V = U for modes of real time series, the f_low cut, and the full row set
against numpy's inverse FFT of the weighted product."""
import numpy as np

import synth


def test_injection_identity(orc):
    data, psd, modes, f = synth.fd_inputs(1, n_det=2, n_modes=3, N=2048, df=0.5, f_low=20.0, noise=False)
    N, df = f.size, 0.5
    fsamp = N * df
    n0 = 357
    rng = np.random.default_rng(2)
    c = rng.normal(size=(2, 3)) + 1j * rng.normal(size=(2, 3))
    shift = np.exp(-2j * np.pi * f * n0 / fsamp)
    data = np.array([(c[k][:, None] * modes).sum(axis=0) * shift for k in range(2)])
    Q, U, V = orc.quv(data, psd, modes, df, 20.0, n0 - 5, 11)
    for k in range(2):
        assert np.abs(Q[k, 5] - U[k] @ c[k]).max() < 1e-10 * np.abs(U[k] @ c[k]).max()
        # the peak of |Q| over the rows is at t0 for a single mode
    _, U1, _ = orc.quv(modes[:1] * shift, psd[:1], modes[:1], df, 20.0, 0, 1)
    Qs, _, _ = orc.quv(modes[:1] * shift, psd[:1], modes[:1], df, 20.0, n0 - 8, 17)
    assert int(np.argmax(np.abs(Qs[0, :, 0]))) == 8
    assert abs(Qs[0, 8, 0] - U1[0, 0, 0]) < 1e-10 * abs(U1[0, 0, 0])


def test_gram_structure(orc):
    data, psd, modes, f = synth.fd_inputs(3, n_det=2, n_modes=4, N=1024, df=1.0, f_low=15.0)
    _, U, V = orc.quv(data, psd, modes, 1.0, 15.0, 0, 1)
    for k in range(2):
        assert np.abs(U[k] - U[k].conj().T).max() < 1e-12 * np.abs(U[k]).max()
        assert np.linalg.eigvalsh(U[k]).min() > -1e-10 * np.abs(U[k]).max()
        assert np.abs(V[k] - V[k].T).max() < 1e-12 * np.abs(V[k]).max()
        # direct sums, written out again from the definition
        w = np.where(np.abs(f) > 15.0, 2.0 / psd[k], 0.0)
        neg = (-np.arange(f.size)) % f.size
        assert np.abs(U[k] - (modes.conj() * w) @ modes.T).max() < 1e-10 * np.abs(U[k]).max()
        assert np.abs(V[k] - (modes[:, neg] * w) @ modes.T).max() < 1e-10 * np.abs(V[k]).max()


def test_real_modes_give_V_equal_U(orc):
    data, psd, modes, f = synth.fd_inputs(4, n_det=1, n_modes=3, N=1024, df=1.0, f_low=15.0)
    neg = (-np.arange(f.size)) % f.size
    real_modes = 0.5 * (modes + modes[:, neg].conj())  # spectra of real time series
    psd_sym = 0.5 * (psd + psd[:, neg])
    _, U, V = orc.quv(data, psd_sym, real_modes, 1.0, 15.0, 0, 1)
    assert np.abs(V - U).max() < 1e-10 * np.abs(U).max()


def test_f_low_cut_and_inverse_fft(orc):
    N, df, fl = 512, 1.0, 30.0
    data, psd, modes, f = synth.fd_inputs(5, n_det=1, n_modes=2, N=N, df=df, f_low=10.0)
    Q, _, _ = orc.quv(data, psd, modes, df, fl, 0, N)
    w = np.where(np.abs(f) > fl, 2.0 * df / psd[0], 0.0)
    for m in range(2):
        ref = N * np.fft.ifft(w * modes[m].conj() * data[0])
        assert np.abs(Q[0, :, m] - ref).max() < 1e-10 * np.abs(ref).max()
    # data inside the cut does not matter
    d2 = data.copy()
    d2[0, np.abs(f) <= fl] += 1e3
    Q2, _, _ = orc.quv(d2, psd, modes, df, fl, 0, 16)
    assert np.abs(Q2 - Q[:, :16]).max() == 0.0


def test_overlaps_give_the_likelihood_peak(orc):
    """The overlaps feed the decomposed likelihood (App. D Eq. (def:lnL:Decomposed)):
    noise-free data h_k(t) = Re[(D_ref/D) F_k sum_m Y_m h_m(t - t_inj)] in one
    detector at the geocentre, Q/U/V of it, and a one-sample window at t_inj:
    ln L_t at the injected parameters equals <h|h>/2, the noise-free maximum
    (App. D.1), with the V term of these complex modes included."""
    N, df, fl = 4096, 0.5, 20.0
    _, psd, modes, f = synth.fd_inputs(11, n_det=1, n_modes=3, N=N, df=df, f_low=fl, noise=False)
    x, yv = np.array(synth.DETECTORS["H1"]["xarm"]), np.array(synth.DETECTORS["H1"]["yarm"])
    P, n_t, n_inj = 4, 1, 1800
    point = dict(Q=np.zeros((1, n_t + 2 * P + 3, 3)), U=np.eye(3)[None], V=None, det_pos=np.zeros((1, 3)),
                 det_resp=(0.5 * (np.outer(x, x) - np.outer(yv, yv)))[None], ell=np.array([2, 2, 3], dtype=np.int32),
                 em=np.array([2, -2, 3], dtype=np.int32), n_t=n_t, pad=P, f_s=N * df, d_ref=100.0, gmst=0.7)
    th = np.array([1.1, -0.4, 0.3, 0.8, 2.0, 180.0, 0.0])
    a = orc.coeffs(orc.Point.from_dict(point), th)[0][0]
    neg = (-np.arange(N)) % N
    s = (a[:, None] * modes).sum(axis=0)
    dtil = 0.5 * (s + s[neg].conj()) * np.exp(-2j * np.pi * f * n_inj / (N * df))
    rho2 = float(np.sum(np.where(np.abs(f) > fl, 2 * df * np.abs(dtil) ** 2 / psd[0], 0.0)))
    Q, U, V = orc.quv(dtil[None], psd, modes, df, fl, n_inj - P - 1, n_t + 2 * P + 3)
    assert np.abs(V).max() > 1e-3 * np.abs(U).max()  # the V term matters here
    point.update(Q=Q, U=U, V=V)
    assert abs(orc.lnL_t(orc.Point.from_dict(point), th) - rho2 / 2) < 1e-10 * rho2
