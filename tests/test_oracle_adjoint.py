"""Pins of the oracle's hand-written adjoints: central finite differences in FP64, the dot-product
test of the linear multislice map, and an independent PyTorch-CPU autograd implementation (built on
torch.fft, not on the oracle's dense DFTs)."""
import math
from types import SimpleNamespace

import numpy as np
import pytest
import torch

from oracle import adjoint as adj
from oracle import multislice as ms
from oracle import potential as pot
from oracle import spectrum as sp
from oracle.physics import interaction_parameter, wavelength, TWO_PI_A0_E, n_segments
from workloads import form_factor_table


def _problem(probe=False, seed=0):
    rng = np.random.default_rng(seed)
    spec = SimpleNamespace(nx=16, ny=16, lx=6.0, ly=5.0, dz=np.array([2.0, 2.0, 2.0]), z0=0.0,
                           bandlimit=2.0 / 3.0)
    n_at, T = 12, 8
    base = np.column_stack([rng.uniform(0, 6, n_at), rng.uniform(0, 5, n_at),
                            rng.choice([0.7, 2.9, 5.1], n_at)])
    pos = (base[None] + 0.15 * rng.normal(size=(T, n_at, 3)) * [1, 1, 0]).astype(np.float32)
    species = rng.integers(0, 2, n_at).astype(np.int32)
    ff = form_factor_table(["A", "B"])
    if probe:
        beam = SimpleNamespace(probe=True, energy_ev=100e3, alpha_rad=0.05, defocus_a=0.0,
                               cs_a=0.0, probe_xy=np.array([[2.0, 2.5], [3.5, 1.0]]))
    else:
        beam = SimpleNamespace(probe=False, energy_ev=100e3)
    n_e, hop, dt, temp = 4, 2, 5.0, 300.0
    emask = adj.energy_filter_mask(n_e, dt, 0.0, 0.2)
    target = rng.uniform(0, 0.02, size=(spec.ny, spec.nx))
    return dict(spec=spec, pos=pos, species=species, ff=ff, beam=beam, n_e=n_e, hop=hop, dt=dt,
                temp=temp, emask=emask, target=target)


def _loss_from_V(pb, V):
    ex = ms.exit_waves(V, pb["spec"], pb["beam"])
    S, _ = sp.spectrum(ex, pb["n_e"], pb["hop"], pb["dt"], pb["temp"])
    return adj.filtered_loss(S, pb["target"], pb["emask"])[0]


def _loss_from_pos(pb, pos):
    V, _ = pot.potentials(pos, pb["species"], pb["ff"], pb["spec"])
    return _loss_from_V(pb, V)


@pytest.mark.parametrize("probe", [False, True])
def test_gradient_wrt_potentials_matches_central_fd(probe):
    pb = _problem(probe, seed=1)
    out = adj.pipeline_gradient(pb["pos"], pb["species"], pb["ff"], pb["spec"], pb["beam"],
                                pb["n_e"], pb["hop"], pb["dt"], pb["temp"], pb["target"],
                                pb["emask"])
    rng = np.random.default_rng(2)
    h = 1e-4
    for _ in range(4):
        d = rng.normal(size=out["V"].shape)
        fd = (_loss_from_V(pb, out["V"] + h * d) - _loss_from_V(pb, out["V"] - h * d)) / (2 * h)
        an = float(np.sum(out["gV"] * d))
        assert an == pytest.approx(fd, rel=1e-6, abs=1e-12 * abs(out["loss"]) + 1e-14)


def test_gradient_wrt_positions_matches_central_fd():
    pb = _problem(False, seed=3)
    out = adj.pipeline_gradient(pb["pos"], pb["species"], pb["ff"], pb["spec"], pb["beam"],
                                pb["n_e"], pb["hop"], pb["dt"], pb["temp"], pb["target"],
                                pb["emask"])
    rng = np.random.default_rng(4)
    h = 1e-4
    pos64 = pb["pos"].astype(np.float64)
    for _ in range(3):
        d = np.zeros(pos64.shape)
        d[..., :2] = rng.normal(size=pos64.shape[:-1] + (2,))
        lp = _loss_from_pos(pb, pos64 + h * d)
        lm = _loss_from_pos(pb, pos64 - h * d)
        fd = (lp - lm) / (2 * h)
        an = float(np.sum(out["gxy"] * d[..., :2]))
        assert an == pytest.approx(fd, rel=1e-6)
    # single coordinates
    for (t, j, c) in ((0, 3, 0), (5, 7, 1), (7, 0, 1)):
        d = np.zeros(pos64.shape)
        d[t, j, c] = 1.0
        fd = (_loss_from_pos(pb, pos64 + h * d) - _loss_from_pos(pb, pos64 - h * d)) / (2 * h)
        assert out["gxy"][t, j, c] == pytest.approx(fd, rel=1e-5, abs=1e-9 * np.abs(out["gxy"]).max())


def test_multislice_dot_product_identity():
    # <A x, y> = <x, A^H y> for the linear map psi_0 -> phi at fixed potentials
    pb = _problem(False, seed=5)
    V, _ = pot.potentials(pb["pos"][:1], pb["species"], pb["ff"], pb["spec"])
    rng = np.random.default_rng(6)
    x = rng.normal(size=(16, 16)) + 1j * rng.normal(size=(16, 16))
    y = rng.normal(size=(16, 16)) + 1j * rng.normal(size=(16, 16))
    ax = ms.propagate(x, V[0], pb["spec"], 100e3)
    _, ahy = adj.multislice_adjoint(x, V[0], pb["spec"], 100e3, y, return_g_psi0=True)
    lhs = np.vdot(y, ax)
    rhs = np.vdot(ahy, x)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


# ------------------------------------------------------------------------------------------
# independent PyTorch-CPU complex128 implementation of the forward pipeline

def _torch_pipeline(pb, pos_xy, V_override=None):
    spec, beam = pb["spec"], pb["beam"]
    nx, ny, lx, ly = spec.nx, spec.ny, spec.lx, spec.ly
    kx = torch.fft.fftfreq(nx, d=lx / nx, dtype=torch.float64)
    ky = torch.fft.fftfreq(ny, d=ly / ny, dtype=torch.float64)
    k2 = ky[:, None] ** 2 + kx[None, :] ** 2
    kn = min(nx / (2 * lx), ny / (2 * ly))
    mask = (k2 < (spec.bandlimit * kn) ** 2).to(torch.float64)
    bins = pot.bin_atoms(pb["pos"][0, :, 2], pot.slice_boundaries(0.0, spec.dz))
    T = pos_xy.shape[0]
    S = len(spec.dz)
    ff = torch.from_numpy(pb["ff"])

    def fz(z):
        q2 = k2
        r = torch.zeros_like(q2)
        for i in range(3):
            r = r + ff[z, 2 * i] / (q2 + ff[z, 2 * i + 1]) + ff[z, 6 + 2 * i] * torch.exp(-ff[z, 7 + 2 * i] * q2)
        return r
    Vs = []
    for t in range(T):
        vt = []
        for s in range(S):
            vk = torch.zeros((ny, nx), dtype=torch.complex128)
            for j in np.nonzero(bins == s)[0]:
                ph = kx[None, :] * pos_xy[t, j, 0] + ky[:, None] * pos_xy[t, j, 1]
                vk = vk + fz(int(pb["species"][j])) * torch.exp(-2j * math.pi * ph)
            vk = vk * mask * (TWO_PI_A0_E / (lx * ly))
            vt.append(torch.fft.ifft2(vk).real * (nx * ny))
        Vs.append(torch.stack(vt))
    V = torch.stack(Vs) if V_override is None else V_override
    lam = wavelength(beam.energy_ev)
    sigma = interaction_parameter(beam.energy_ev)
    exits = []
    for t in range(T):
        psi = torch.full((ny, nx), 1 / math.sqrt(nx * ny), dtype=torch.complex128)
        for s in range(S):
            u = torch.exp(1j * sigma * V[t, s]) * psi
            prop = mask * torch.exp(-1j * math.pi * lam * spec.dz[s] * k2)
            if s < S - 1:
                psi = torch.fft.ifft2(prop * torch.fft.fft2(u))
            else:
                exits.append(prop * torch.fft.fft2(u) / math.sqrt(nx * ny))
    ex = torch.stack(exits)                                        # [T][ny][nx]
    n_e, hop = pb["n_e"], pb["hop"]
    G = n_segments(T, n_e, hop)
    P = sum(torch.abs(torch.fft.fft(ex[g * hop:g * hop + n_e], dim=0)) ** 2 for g in range(G)) / G
    K = torch.from_numpy(sp.kubo_table_dft_order(n_e, pb["dt"], pb["temp"]))
    KP = K[:, None, None] * P
    I = torch.fft.fftshift(KP / KP.sum())
    em = torch.from_numpy(pb["emask"])
    d = I[em].sum(0) - torch.from_numpy(np.fft.fftshift(np.fft.fftshift(pb["target"])))
    return (d ** 2).sum(), V


def test_hand_adjoint_matches_torch_autograd():
    pb = _problem(False, seed=7)
    out = adj.pipeline_gradient(pb["pos"], pb["species"], pb["ff"], pb["spec"], pb["beam"],
                                pb["n_e"], pb["hop"], pb["dt"], pb["temp"], pb["target"],
                                pb["emask"])
    xy = torch.tensor(pb["pos"][..., :2].astype(np.float64), requires_grad=True)
    loss, V = _torch_pipeline(pb, xy)
    V.retain_grad()
    loss.backward()
    assert float(loss) == pytest.approx(out["loss"], rel=1e-10)
    np.testing.assert_allclose(V.detach().numpy(), out["V"], atol=1e-10 * np.abs(out["V"]).max())
    np.testing.assert_allclose(V.grad.numpy(), out["gV"], atol=1e-9 * np.abs(out["gV"]).max())
    np.testing.assert_allclose(xy.grad.numpy(), out["gxy"], atol=1e-9 * np.abs(out["gxy"]).max())
