"""Edge cases of the hot path through the C ABI, against the FP64 oracle.

Single-slice specimens, slices without atoms, the smallest (16^2) and largest (1024^2) grids, the
longest time segment (n_e = 1024), a trajectory that is exactly one segment long, and argument
errors that must be reported before any launch.
"""
from types import SimpleNamespace

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

import paper_2401_15599_amd as tw
from oracle import multislice as o_ms
from oracle import potential as o_pot
from oracle import spectrum as o_sp
from workloads import form_factor_table

DEV = "cuda:0"


def rel_l2(a, b):
    return float(np.linalg.norm((np.asarray(a) - b).ravel()) / np.linalg.norm(np.asarray(b).ravel()))


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _specimen(n, lx, dz, n_atoms, T, seed, z_hi=None):
    rng = np.random.default_rng(seed)
    zt = float(np.sum(dz)) if z_hi is None else z_hi
    pos = np.stack([rng.uniform(0, lx, (T, n_atoms)), rng.uniform(0, lx, (T, n_atoms)),
                    rng.uniform(0, zt, (T, n_atoms))], axis=-1).astype(np.float32)
    species = rng.integers(0, 2, n_atoms).astype(np.int32)
    spec = SimpleNamespace(nx=n, ny=n, lx=lx, ly=lx, dz=np.asarray(dz, float), z0=0.0,
                           bandlimit=2.0 / 3.0)
    return spec, pos, species


def _pipeline(spec, pos, species, beam, mode=tw.MODE_BATCHED):
    ff = form_factor_table(["A", "B"])
    ctx = tw.context(0)
    T = pos.shape[0]
    V = torch.empty((T, len(spec.dz), spec.ny, spec.nx), dtype=torch.float32, device=DEV)
    tw.tacaw_build_potentials(ctx, tw.specimen_from(spec), _gpu(pos), _gpu(species), ff, V)
    n_pos = beam.probe_xy.shape[0] if beam.probe else 1
    ex = torch.empty((T, n_pos, spec.ny, spec.nx), dtype=torch.complex64, device=DEV)
    ex.fill_(float("nan"))
    tw.tacaw_multislice(ctx, [tw.MsJob(tw.specimen_from(spec), tw.beam_from(beam), V, ex)],
                        mode=mode)
    Vr, _ = o_pot.potentials(pos, species, ff, spec)
    return V.cpu().numpy(), Vr, ex.cpu().numpy()


PLANE = SimpleNamespace(probe=False, energy_ev=100e3)


@pytest.mark.parametrize("mode", [tw.MODE_BATCHED, tw.MODE_PLAIN])
def test_single_slice(mode):
    spec, pos, species = _specimen(64, 16.0, [2.0], 30, 2, 1)
    V, Vr, ex = _pipeline(spec, pos, species, PLANE, mode)
    assert rel_l2(V, Vr) <= 1e-5
    ref = o_ms.exit_waves(Vr.astype(np.float32).astype(np.float64), spec, PLANE)
    assert rel_l2(ex, ref) <= 1e-4


def test_slices_without_atoms():
    # atoms only in the first of four slices: V of the others is exactly zero
    spec, pos, species = _specimen(64, 16.0, [2.0] * 4, 25, 2, 2, z_hi=1.9)
    V, Vr, ex = _pipeline(spec, pos, species, PLANE)
    assert np.all(V[:, 1:] == 0.0)
    assert rel_l2(V, Vr) <= 1e-5
    ref = o_ms.exit_waves(Vr.astype(np.float32).astype(np.float64), spec, PLANE)
    assert rel_l2(ex, ref) <= 1e-4


def test_empty_slice_paired_with_an_occupied_one():
    # band-limited maps are inverse-transformed two at a time (A + iB); an empty map stays exactly
    # zero whichever side of its pair it is on, and an odd map count leaves the last one unpaired
    spec, pos, species = _specimen(128, 24.0, [2.0] * 3, 40, 1, 5)
    pos[..., 2] = np.float32(2.0) + pos[..., 2] % np.float32(2.0) * np.float32(0.5)   # slice 1 only
    V, Vr, _ = _pipeline(spec, pos, species, PLANE)
    assert np.all(V[:, 0] == 0.0) and np.all(V[:, 2] == 0.0)
    assert np.any(V[:, 1] != 0.0)
    assert rel_l2(V, Vr) <= 1e-5


def test_empty_slices_across_snapshot_passes():
    # 1024^2 with 65 slices: the potential build takes one snapshot per pass (its 1 GiB k-space
    # budget), so the second pass starts at snapshot 1 and each pass pairs an odd number of maps;
    # atoms only in the first 10 slices, the other 55 maps exactly zero
    rng = np.random.default_rng(21)
    S, A = 65, 24
    pos = np.stack([rng.uniform(0, 60.0, (2, A)), rng.uniform(0, 60.0, (2, A)),
                    rng.uniform(0, 4.9, (2, A))], axis=-1).astype(np.float32)
    species = rng.integers(0, 2, A).astype(np.int32)
    spec = SimpleNamespace(nx=1024, ny=1024, lx=60.0, ly=60.0, dz=np.full(S, 0.5), z0=0.0,
                           bandlimit=2.0 / 3.0)
    ff = form_factor_table(["A", "B"])
    V = torch.empty((2, S, 1024, 1024), dtype=torch.float32, device=DEV)
    tw.tacaw_build_potentials(tw.context(0), tw.specimen_from(spec), _gpu(pos), _gpu(species), ff, V)
    torch.cuda.synchronize()
    assert bool((V[:, 10:] == 0).all())
    sel = [0, 3, 9]
    Vr, _ = o_pot.potentials(pos, species, ff, SimpleNamespace(**{**vars(spec), "dz": np.full(10, 0.5)}))
    for t in range(2):
        for s in sel:
            assert rel_l2(V[t, s].cpu().numpy(), Vr[t, s]) <= 1e-5, (t, s)


def test_smallest_grid_with_probe():
    spec, pos, species = _specimen(16, 4.0, [1.5, 1.5], 6, 3, 3)
    beam = SimpleNamespace(probe=True, energy_ev=100e3, alpha_rad=0.05, defocus_a=10.0, cs_a=0.0,
                           probe_xy=np.array([[1.0, 2.0], [3.1, 0.4]]))
    V, Vr, ex = _pipeline(spec, pos, species, beam)
    assert rel_l2(V, Vr) <= 1e-5
    ref = o_ms.exit_waves(Vr.astype(np.float32).astype(np.float64), spec, beam)
    assert rel_l2(ex, ref) <= 1e-4


def test_largest_grid():
    # 1024^2: the x pass and the y pass take the 16-element plans (the y pass as the block kernel
    # on 512 threads)
    spec, pos, species = _specimen(1024, 320.0, [2.0, 2.0], 400, 1, 4)
    V, Vr, ex = _pipeline(spec, pos, species, PLANE)
    assert rel_l2(V, Vr) <= 1e-5
    ref = o_ms.exit_waves(Vr.astype(np.float32).astype(np.float64), spec, PLANE)
    assert rel_l2(ex, ref) <= 1e-4


def test_longest_segment_single_segment_trajectory():
    rng = np.random.default_rng(9)
    T, P, n = 1024, 1, 16
    ex = (rng.normal(size=(T, P, n, n)) + 1j * rng.normal(size=(T, P, n, n))).astype(np.complex64)
    opts = tw.SpectrumOpts(2.0, 300.0, 1024, 1024, n, n)
    S = torch.empty((1024, n, n), dtype=torch.float32, device=DEV)
    norm = torch.empty((1,), dtype=torch.float64, device=DEV)
    tw.tacaw_autocorr_spectrum(tw.context(0), _gpu(ex), opts, S, norm)
    ref, Z = o_sp.spectrum(ex.astype(np.complex128), 1024, 1024, 2.0, 300.0, n, n)
    assert rel_l2(S.cpu().numpy(), ref) <= 1e-3
    assert abs(norm.item() - Z) <= 1e-5 * Z


def test_argument_errors_leave_outputs_untouched():
    ctx = tw.context(0)
    spec, pos, species = _specimen(64, 16.0, [2.0], 10, 1, 5)
    V = torch.zeros((1, 1, 64, 64), dtype=torch.float32, device=DEV)
    ex = torch.full((1, 1, 64, 64), 7.0, dtype=torch.complex64, device=DEV)
    bad = tw.specimen_from(spec)
    bad.nx = 48                                   # not a power of two
    with pytest.raises(tw.TacawError):
        tw.tacaw_multislice(ctx, [tw.MsJob(bad, tw.Beam(100e3), V, ex)])
    assert torch.all(ex == 7.0)
    opts = tw.SpectrumOpts(5.0, 300.0, 16, 4, 64, 64)
    with pytest.raises(tw.TacawError):             # segment longer than the trajectory
        tw.tacaw_autocorr_spectrum(ctx, ex, opts, torch.empty((16, 64, 64), device=DEV))
