"""The five synthetic workloads and their small test variants.

Each entry states the cell, grid, slicing, beam, trajectory and spectrum parameters of one
workload.  Unstated parameters follow these choices: dt = 5 fs where the workload gives none,
100 keV beams where none is given, one energy segment (N_E = T) where none is given,
T = 300 K throughout (the temperature of the paper's experiments), band limit 2/3 of the
smaller Nyquist frequency.

`make_workload(name)` returns a `Workload` with every array a consumer needs; the same object
feeds the CPU oracle and the GPU library.
"""
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from .formfactors import form_factor_table
from .structures import bcc_cubic, diamond_cubic, fcc_cubic, hexagonal_bn_like, rocksalt
from .trajectory import harmonic_trajectory


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    lx: float
    ly: float
    dz: np.ndarray                 # float64 [S] slice thicknesses
    z0: float
    energy_ev: float
    probe: bool
    alpha_rad: float
    defocus_a: float
    cs_a: float
    probe_xy: np.ndarray           # float64 [P][2]
    bandlimit: float
    dt_fs: float
    n_snap: int
    n_e: int
    hop: int
    temperature_k: float
    nqx_out: int
    nqy_out: int
    positions: Optional[np.ndarray]  # float32 [T][N][3] (None until generated)
    species: np.ndarray            # int32 [N]
    ff: np.ndarray                 # float64 [n_species][12]
    seed: int
    extra: dict = field(default_factory=dict)

    @property
    def n_slices(self):
        return int(self.dz.shape[0])

    @property
    def n_pos(self):
        return int(self.probe_xy.shape[0])


def _probe_grid(center_xy, n=8, step=0.5):
    off = (np.arange(n) - (n - 1) / 2.0) * step
    gx, gy = np.meshgrid(center_xy[0] + off, center_xy[1] + off, indexing="xy")
    return np.stack([gx.ravel(), gy.ravel()], axis=1).astype(np.float64)


CONFIGS = {
    # configs[0]: tiny plain method
    "c1": dict(kind="fcc", a=4.0, reps=(4, 4, 4), n=(64, 64), n_slices=4, dz=4.0,
               energy=100e3, T=32, dt=5.0, n_e=32, hop=32, seed=1001),
    "c1-seg": dict(kind="fcc", a=4.0, reps=(4, 4, 4), n=(64, 64), n_slices=4, dz=4.0,
                   energy=100e3, T=32, dt=5.0, n_e=16, hop=8, seed=1001),
    # configs[1]: plain single specimen, full S(q, omega) on the 256^2 q grid, 256 bins
    "c2": dict(kind="rocksalt", a=4.0, reps=(10, 10, 20), n=(256, 256), n_slices=40, dz=2.0,
               energy=100e3, T=512, dt=5.0, n_e=256, hop=128, seed=2001),
    # configs[3]: differentiation, hexagonal B/N-like stack
    "c4": dict(kind="hbn", a=2.50, c=6.66, reps=(16, 9, 10), n=(256, 256), n_slices=20,
               dz=3.33, energy=100e3, T=128, dt=5.0, n_e=128, hop=128, seed=4001,
               omega_a=130.0, omega_o=170.0),
    # configs[4]: large hexagonal stack (generated only at reduced size in tests)
    "c5": dict(kind="hbn", a=2.50, c=6.66, reps=(40, 40, 50), n=(1024, 1024), n_slices=100,
               dz=3.33, energy=60e3, T=2048, dt=2.0, n_e=1024, hop=512, seed=5001,
               omega_a=130.0, omega_o=170.0),
}


def c3_specimens():
    """configs[2]: 24 rocksalt specimens, 8 per grid class, slices 10..80 of 2 Angstrom.

    All classes use 0.3125 Angstrom pixels; the probe (100 keV, 30 mrad, Cs = 0, no defocus)
    is scanned over 8 x 8 positions on a 0.5 Angstrom grid covering one unit cell near the
    cell centre.
    """
    out = []
    seed = 3001
    for n, cells in ((128, 10), (256, 20), (512, 40)):
        for s in range(10, 81, 10):
            out.append(dict(kind="rocksalt", a=4.0, reps=(cells, cells, s // 2), n=(n, n),
                            n_slices=s, dz=2.0, energy=100e3, T=256, dt=5.0, n_e=256, hop=256,
                            seed=seed, probe=True, alpha=0.030))
            seed += 1
    return out


def _structure(cfg):
    if cfg["kind"] == "fcc":
        return fcc_cubic(cfg["a"], cfg["reps"])
    if cfg["kind"] == "rocksalt":
        return rocksalt(cfg["a"], cfg["reps"])
    if cfg["kind"] == "hbn":
        return hexagonal_bn_like(cfg["a"], cfg["c"], cfg["reps"])
    if cfg["kind"] == "diamond":
        return diamond_cubic(cfg["a"], cfg["reps"])
    if cfg["kind"] == "bcc":
        return bcc_cubic(cfg["a"], cfg["reps"])
    raise ValueError(cfg["kind"])


def make_workload(cfg, n_snap=None, generate=True, device=None, name=None, **over):
    """Build a Workload from a config dict (or a key of CONFIGS).

    `n_snap` truncates the trajectory (the first n_snap snapshots of the same seeded run);
    `over` overrides scalar fields (e.g. n_e, hop, nqx_out).
    """
    if isinstance(cfg, str):
        name = name or cfg
        cfg = CONFIGS[cfg]
    cfg = dict(cfg)
    cfg.update({k: v for k, v in over.items() if k in cfg})
    st = _structure(cfg)
    nx, ny = cfg["n"]
    lx, ly, lz = st.cell
    s = cfg["n_slices"]
    dz = np.full(s, float(cfg["dz"]))
    T = int(n_snap if n_snap is not None else cfg["T"])
    probe = bool(cfg.get("probe", False))
    if probe:
        pxy = _probe_grid((lx / 2.0, ly / 2.0))
    else:
        pxy = np.zeros((1, 2))
    pos = None
    if generate:
        pos = harmonic_trajectory(st, T, cfg["dt"], cfg["seed"],
                                  omega_a_mev=cfg.get("omega_a", 35.0),
                                  omega_o_mev=cfg.get("omega_o", 60.0), device=device)
    n_e = int(over.get("n_e", min(cfg["n_e"], T)))
    hop = int(over.get("hop", min(cfg["hop"], T)))
    return Workload(
        name=name or cfg.get("name", cfg["kind"]), nx=nx, ny=ny, lx=lx, ly=ly, dz=dz,
        z0=0.0, energy_ev=float(cfg["energy"]), probe=probe,
        alpha_rad=float(cfg.get("alpha", 0.0)), defocus_a=0.0, cs_a=0.0, probe_xy=pxy,
        bandlimit=float(over.get("bandlimit", 2.0 / 3.0)), dt_fs=float(cfg["dt"]), n_snap=T,
        n_e=n_e, hop=hop, temperature_k=float(over.get("temperature_k", 300.0)),
        nqx_out=int(over.get("nqx_out", nx)), nqy_out=int(over.get("nqy_out", ny)),
        positions=pos, species=st.species.astype(np.int32),
        ff=form_factor_table(st.species_names), seed=int(cfg["seed"]),
        extra=dict(structure=st, lz=lz))
