"""The single-specimen, differentiation and large workloads at their full sizes, checked against the
FP64 oracle on everything it can afford: whole arrays where its dense transforms finish in seconds,
sampled snapshots and slices otherwise, and properties that hold at any size for the rest.

* rocksalt 10x10x20 cells, 256^2, 40 slices, 100 keV plane wave, 512 snapshots, S(q, w) with 256
  bins and hop 128: every potential of one snapshot, its exit wave, and the whole spectrum of the
  device's exit stack;
* B/N-like 16x9x10 cells, 256^2, 20 slices, 128 snapshots, loss on the 0-200 meV filtered
  diffraction: the loss, dL/dV of two snapshots and their atoms' dL/d(x, y), from the oracle's
  adjoint chain applied to the device's forward intermediates;
* B/N-like 40x40x50 cells (640,000 atoms), 1024^2, 100 slices, 60 keV, 2048 snapshots streamed in
  chunks (17 GB of exit waves), 1024 energy bins: two sampled slice potentials, a three-slice
  multislice of a sampled snapshot, the periodogram at 48 sampled q, and norm/finite/sum rules
  over everything.
"""
import math

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

import paper_2401_15599_amd as tw
from paper_2401_15599_amd.autograd import TacawMultislice, TacawPotentials, TacawSpectrum
from oracle import adjoint as o_adj
from oracle import multislice as o_ms
from oracle import potential as o_pot
from oracle import spectrum as o_sp
from workloads import make_workload

DEV = "cuda:0"


def rel_l2(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def check(a, b, tol, what):
    e = rel_l2(a, b)
    assert e <= tol, f"{what}: rel-L2 {e:.3e} > {tol:g}"


def _norms(ex, chunk=128):
    """sum |phi|^2 of every wave of an exit stack [T][P][ny][nx], chunked; also checks finiteness."""
    out = []
    for t0 in range(0, ex.shape[0], chunk):
        e = ex[t0:t0 + chunk]
        assert bool(torch.isfinite(torch.view_as_real(e)).all()), f"non-finite exit waves at {t0}"
        out.append((e.real.double() ** 2 + e.imag.double() ** 2).sum(dim=(2, 3)).cpu().numpy())
    return np.concatenate(out)


def test_single_specimen_full_size():
    w = make_workload("c2")
    T, S = w.n_snap, w.n_slices
    cx = tw.context(0)
    sp, bm = tw.specimen_from(w), tw.beam_from(w)
    V = torch.empty((T, S, w.ny, w.nx), dtype=torch.float32, device=DEV)
    tw.tacaw_build_potentials(cx, sp, torch.from_numpy(w.positions).to(DEV),
                              torch.from_numpy(w.species).to(DEV), w.ff, V)
    ex = torch.empty((T, 1, w.ny, w.nx), dtype=torch.complex64, device=DEV)
    tw.tacaw_multislice(cx, [tw.MsJob(sp, bm, V, ex)], mode=tw.MODE_BATCHED)
    opts = tw.SpectrumOpts(w.dt_fs, 300.0, w.n_e, w.hop, w.nx, w.ny)
    Sq = torch.empty((w.n_e, w.ny, w.nx), dtype=torch.float32, device=DEV)
    norm = torch.empty((1,), dtype=torch.float64, device=DEV)
    tw.tacaw_autocorr_spectrum(cx, ex, opts, Sq, norm)
    torch.cuda.synchronize()

    t = 200
    V_ref, _ = o_pot.potentials(w.positions[t:t + 1], w.species, w.ff, w)
    check(V[t].cpu().numpy(), V_ref[0], 1e-5, f"potentials of snapshot {t}")
    Vt = V[t:t + 1].cpu().numpy().astype(np.float64)
    check(ex[t].cpu().numpy(), o_ms.exit_waves(Vt, w, w)[0], 1e-4, f"exit wave of snapshot {t}")
    n = _norms(ex)
    assert np.all(n > 0.5) and np.all(n <= 1.0 + 1e-4), (n.min(), n.max())
    ex_host = ex.cpu().numpy().astype(np.complex128)
    S_ref, Z = o_sp.spectrum(ex_host, w.n_e, w.hop, w.dt_fs, 300.0)
    check(Sq.cpu().numpy(), S_ref, 1e-3, "spectrum of the exit stack")
    assert abs(norm.item() - Z) <= 1e-5 * Z


def test_differentiation_workload_full_size_sampled():
    w = make_workload("c4")
    T, S = w.n_snap, w.n_slices
    stride = math.ceil(math.sqrt(S))
    rng = np.random.default_rng(4001)
    target = rng.uniform(0.0, 2.0 / (w.nx * w.ny), size=(w.ny, w.nx))
    emask = o_adj.energy_filter_mask(w.n_e, w.dt_fs, 0.0, 0.2)
    tspec, tbeam = tw.specimen_from(w), tw.beam_from(w)
    xyz = torch.from_numpy(w.positions).to(DEV).requires_grad_(True)
    V = TacawPotentials.apply(xyz, torch.from_numpy(w.species).to(DEV), tspec, w.ff)
    V.retain_grad()
    ex = TacawMultislice.apply(V, tspec, tbeam, stride)
    ex.retain_grad()
    Sq = TacawSpectrum.apply(ex, tw.SpectrumOpts(w.dt_fs, 300.0, w.n_e, w.hop, w.nx, w.ny))
    em = torch.from_numpy(emask).to(DEV)
    tg = torch.from_numpy(target.astype(np.float32)).to(DEV)
    loss = ((Sq[em].sum(0) - tg) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()

    # the oracle's adjoint chain from the device's forward intermediates
    ex_host = ex.detach().cpu().numpy().astype(np.complex128)
    S_ref, _ = o_sp.spectrum(ex_host, w.n_e, w.hop, w.dt_fs, 300.0)
    loss_ref, gS = o_adj.filtered_loss(S_ref, target, emask)
    assert abs(loss.item() - loss_ref) <= 1e-3 * loss_ref
    g_ex = o_adj.spectrum_backward(ex_host, gS, w.n_e, w.hop, w.dt_fs, 300.0)
    check(ex.grad.cpu().numpy(), g_ex, 1e-3, "dL/dphi")
    psi0 = o_ms.initial_waves(w, w)
    for t in (0, 77):
        Vt = V[t].detach().cpu().numpy().astype(np.float64)
        gV = o_adj.multislice_adjoint(psi0[0], Vt, w, w.energy_ev, g_ex[t, 0])
        check(V.grad[t].cpu().numpy(), gV, 1e-3, f"dL/dV of snapshot {t}")
        gxy = o_adj.position_gradient(gV, w.positions[t], w.species, w.ff, w)
        check(xyz.grad[t, :, :2].cpu().numpy(), gxy, 1e-3, f"dL/dxy of snapshot {t}")
    assert float(xyz.grad[..., 2].abs().max()) == 0.0


def test_large_workload_full_size_sampled():
    import bench
    r = bench.large_run(tw, keep=True)
    d = r.pop("tensors")
    w, ex, V, P, Sq, norm = d["w"], d["exit"], d["V"], d["P"], d["S"], d["norm"]
    T, S = w.n_snap, w.n_slices
    xyz = d["xyz"]
    del d
    # every exit wave finite, norms in (0.5, 1] (the band limit only removes intensity)
    n = _norms(ex)
    assert np.all(n > 0.5) and np.all(n <= 1.0 + 1e-4), (n.min(), n.max())
    # two slices of a snapshot of the last chunk, from its atoms alone
    ts = T - 3
    idx = ts - (T - 1) // 64 * 64
    pos = xyz[ts].cpu().numpy()
    bins = o_pot.bin_atoms(pos[:, 2].astype(np.float64), o_pot.slice_boundaries(w.z0, w.dz))
    mask = o_pot.bandlimit_mask(w.nx, w.ny, w.lx, w.ly, w.bandlimit)
    for s in (0, 61):
        sel = bins == s
        ref = o_pot.slice_potential(pos[sel, :2].astype(np.float64), w.species[sel], w.ff, w.nx,
                                    w.ny, w.lx, w.ly, mask)
        check(V[idx, s].cpu().numpy(), ref, 1e-5, f"potential of slice {s}, snapshot {ts}")
    # the first three slices of that snapshot through the device and the oracle
    V3 = V[idx:idx + 1, :3].contiguous()
    w3 = make_workload("c5", generate=False)
    w3.dz = w.dz[:3]
    out = torch.empty((1, 1, w.ny, w.nx), dtype=torch.complex64, device=DEV)
    tw.tacaw_multislice(tw.context(0), [tw.MsJob(tw.specimen_from(w3), tw.beam_from(w3), V3, out)])
    ref = o_ms.exit_waves(V3.cpu().numpy().astype(np.float64), w3, w3)[0, 0]
    check(out[0, 0].cpu().numpy(), ref, 1e-4, "three-slice wave at 1024^2")
    # periodogram at 48 sampled q from the device's exit stack
    rng = np.random.default_rng(5)
    qy, qx = rng.integers(0, w.ny, 48), rng.integers(0, w.nx, 48)
    cols = ex[:, 0, torch.from_numpy(qy).to(DEV), torch.from_numpy(qx).to(DEV)]      # [T][48]
    stack = cols.cpu().numpy().astype(np.complex128)[:, None, None, :]
    P_ref = o_sp.segment_periodogram(stack, w.n_e, w.hop)[:, 0, :]                   # [n_e][48]
    P_got = P[:, torch.from_numpy(qy).to(DEV), torch.from_numpy(qx).to(DEV)].cpu().numpy()
    check(P_got, P_ref, 1e-3, "periodogram at sampled q")
    # the spectrum sums to one and its normalisation is the Kubo-weighted periodogram total
    assert abs(float(Sq.double().sum().item()) - 1.0) < 1e-3
    K = torch.from_numpy(o_sp.kubo_table_dft_order(w.n_e, w.dt_fs, w.temperature_k)).to(DEV)
    Z = float((P.double().sum(dim=(1, 2)) * K).sum().item())
    assert abs(norm.item() - Z) <= 1e-5 * Z
