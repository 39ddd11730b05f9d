"""Seeded synthetic trajectories: superpositions of harmonic phonon-like modes.

u_j(t) = sum_m a_m s_mj e_m cos(2 pi Q_m . R_j - omega_m t + theta_m)

* Q_m: random wave vectors allowed by the periodic supercell, (h/Lx, k/Ly, l/Lz).
* theta_m ~ U[0, 2 pi); e_m is longitudinal (along Q_m) for half the modes, random otherwise.
* The first half of the modes is acoustic, s_mj = +1 and omega = omega_A |sin(pi a |Q| / 2)|
  (floored at 2 meV); the second half is optical, s_mj = -1 on the second species and
  omega = omega_O (1 - 0.1 cos(pi a |Q|)).
* a_m proportional to 1/omega_m (equipartition), rescaled so that the RMS displacement per
  Cartesian component is `rms` (0.07 Angstrom by default).

Time is t_n = n * dt.  The output is float32 [T][N][3] in Angstrom, like a stored MD trajectory.
"""
import numpy as np

HBAR_MEV_FS = 658.2119569  # hbar in meV*fs (used only to turn mode energies into angular frequencies)


def _modes(struct, n_modes, omega_a_mev, omega_o_mev, rms, rng):
    lx, ly, lz = struct.cell
    ncell = np.maximum(1, np.round(np.array(struct.cell) / struct.lattice_a)).astype(int)
    h = rng.integers(-(ncell // 2), ncell // 2 + 1, size=(n_modes, 3))
    q = h / np.array([lx, ly, lz])                                   # 1/Angstrom
    qn = np.linalg.norm(q, axis=1)
    theta = rng.uniform(0.0, 2.0 * np.pi, size=n_modes)
    rand_dir = rng.normal(size=(n_modes, 3))
    rand_dir /= np.linalg.norm(rand_dir, axis=1, keepdims=True)
    e = rand_dir.copy()
    half = n_modes // 2
    lon = np.arange(n_modes) % 2 == 0                                # alternate longitudinal / random
    with np.errstate(invalid="ignore", divide="ignore"):
        qhat = np.where(qn[:, None] > 0, q / qn[:, None], rand_dir)
    e[lon] = qhat[lon]
    optical = np.arange(n_modes) >= half
    a = struct.lattice_a
    w_ac = np.maximum(omega_a_mev * np.abs(np.sin(np.pi * a * qn / 2.0)), 2.0)
    w_op = omega_o_mev * (1.0 - 0.1 * np.cos(np.pi * a * qn))
    e_mev = np.where(optical, w_op, w_ac)
    omega = e_mev / HBAR_MEV_FS                                      # rad/fs
    amp = 1.0 / omega
    amp *= rms / np.sqrt(np.sum(amp ** 2) / 6.0)                     # <cos^2>=1/2, 1/3 per component
    return q, theta, e, optical, omega, amp


def harmonic_trajectory(struct, n_snap, dt_fs, seed, n_modes=256, omega_a_mev=35.0,
                        omega_o_mev=60.0, rms=0.07, device=None, atom_chunk=1 << 16):
    """Generate positions float32 [n_snap][N][3].

    With `device` set to a torch device the large time-by-mode product runs there (used only for
    benchmark-scale inputs); otherwise NumPy float64 is used.  Mode parameters always come from
    NumPy's seeded generator, so the two routes describe the same trajectory.
    """
    rng = np.random.default_rng(seed)
    q, theta, e, optical, omega, amp = _modes(struct, n_modes, omega_a_mev, omega_o_mev, rms, rng)
    r0 = struct.positions
    n = r0.shape[0]
    t = np.arange(n_snap, dtype=np.float64) * dt_fs
    tau = np.exp(-1j * np.outer(t, omega))                              # [T][M]
    second = struct.species == 1
    if device is None:
        out = np.empty((n_snap, n, 3), dtype=np.float32)
    else:
        import torch
        out = torch.empty((n_snap, n, 3), dtype=torch.float32, device=device)
        tau_d = torch.from_numpy(tau.astype(np.complex64)).to(device)
    if device is not None:
        # same arithmetic with torch on the device (float64 phases, complex64 time products)
        qd = torch.from_numpy(q).to(device)
        thd = torch.from_numpy(theta).to(device)
        ampd = torch.from_numpy(amp).to(device)
        optd = torch.from_numpy(optical).to(device)
        ed = torch.from_numpy(e).to(device)
        r0d = torch.from_numpy(r0).to(device)
        secd = torch.from_numpy(second).to(device)
        for j0 in range(0, n, atom_chunk):
            j1 = min(n, j0 + atom_chunk)
            phase = 2.0 * np.pi * (r0d[j0:j1] @ qd.T) + thd[None, :]
            sign = torch.where(optd[None, :] & secd[j0:j1, None], -1.0, 1.0).to(torch.float64)
            coef = torch.complex(torch.cos(phase), torch.sin(phase)) * (ampd[None, :] * sign)
            for c in range(3):
                w = (coef * ed[None, :, c]).T.to(torch.complex64)
                u = (tau_d @ w).real
                out[:, j0:j1, c] = r0d[None, j0:j1, c].float() + u
        return out
    for j0 in range(0, n, atom_chunk):
        j1 = min(n, j0 + atom_chunk)
        phase = 2.0 * np.pi * (r0[j0:j1] @ q.T) + theta[None, :]        # [n][M]
        sign = np.where(optical[None, :] & second[j0:j1, None], -1.0, 1.0)
        coef = (amp[None, :] * sign) * np.exp(1j * phase)               # [n][M]
        for c in range(3):
            w = coef * e[None, :, c]
            u = (tau @ w.T).real                                        # [T][n]
            out[:, j0:j1, c] = (r0[None, j0:j1, c] + u).astype(np.float32)
    return out


def static_trajectory(struct, n_snap):
    """Every snapshot equal to the equilibrium structure (a static lattice)."""
    p = struct.positions.astype(np.float32)
    return np.repeat(p[None], n_snap, axis=0)


def rigid_shift_trajectory(struct, n_snap, pixel_x, seed, max_shift=3):
    """All atoms shifted rigidly along x by an integer number of pixels p(t) per snapshot.

    Returns (positions float32 [T][N][3], shifts int [T]).  The pixel size must make
    p * pixel_x exactly representable (e.g. 0.25 Angstrom) for the shift to be exact.
    """
    rng = np.random.default_rng(seed)
    p = rng.integers(-max_shift, max_shift + 1, size=n_snap)
    pos = np.repeat(struct.positions[None].astype(np.float64), n_snap, axis=0)
    pos[:, :, 0] += p[:, None] * pixel_x
    return pos.astype(np.float32), p
