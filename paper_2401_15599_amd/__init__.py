"""Python binding of the TACAW hot-path library (libtacaw.so, gfx950).

Argument marshalling only: every function below forwards to the C entry point of the same name in
include/tacaw.h, passing device pointers of torch tensors and torch's current HIP stream.  All
arithmetic runs in the library's HIP kernels.  There is no CPU fallback: importing this package
raises if the compiled library is missing, and every call raises TacawError on a non-zero status.
"""
import ctypes
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np
# torch carries its own HIP runtime (soname libamdhip64.so.7).  Loading it before the library makes
# libtacaw bind to that same runtime; the other order puts two HIP runtimes in the process and
# torch then finds no GPU.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtacaw.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2401_15599_amd/build.py`")

_lib = ctypes.CDLL(LIB_PATH)

PLANE_WAVE, PROBE = 0, 1
MODE_PLAIN, MODE_BATCHED, MODE_PERSISTENT = 0, 1, 2


class TacawError(RuntimeError):
    pass


class _Spec(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("lx", ctypes.c_double),
                ("ly", ctypes.c_double), ("n_slices", ctypes.c_int32),
                ("dz", ctypes.POINTER(ctypes.c_double)), ("z0", ctypes.c_double),
                ("bandlimit", ctypes.c_double)]


class _Beam(ctypes.Structure):
    _fields_ = [("energy_ev", ctypes.c_double), ("kind", ctypes.c_int32),
                ("alpha_rad", ctypes.c_double), ("defocus_a", ctypes.c_double),
                ("cs_a", ctypes.c_double), ("n_pos", ctypes.c_int32),
                ("pos_xy", ctypes.POINTER(ctypes.c_double))]


class _Job(ctypes.Structure):
    _fields_ = [("spec", ctypes.POINTER(_Spec)), ("beam", ctypes.POINTER(_Beam)),
                ("n_snap", ctypes.c_int32), ("V", ctypes.c_void_p), ("exit", ctypes.c_void_p),
                ("ckpt", ctypes.c_void_p)]


class KernelStats(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("algo_bytes", ctypes.c_double)]


class _Opts(ctypes.Structure):
    _fields_ = [("dt_fs", ctypes.c_double), ("temperature_k", ctypes.c_double),
                ("n_e", ctypes.c_int32), ("hop", ctypes.c_int32), ("nqx_out", ctypes.c_int32),
                ("nqy_out", ctypes.c_int32)]


_P = ctypes.c_void_p
_I = ctypes.c_int32
_SIGS = {
    "tacaw_version": ([], ctypes.c_int),
    "tacaw_create": ([ctypes.c_int, ctypes.POINTER(_P)], ctypes.c_int),
    "tacaw_destroy": ([_P], None),
    "tacaw_last_error": ([], ctypes.c_char_p),
    "tacaw_wavelength": ([ctypes.c_double], ctypes.c_double),
    "tacaw_interaction_parameter": ([ctypes.c_double], ctypes.c_double),
    "tacaw_energy_axis": ([_I, ctypes.c_double, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "tacaw_bin_atoms": ([_P, ctypes.POINTER(_Spec), _I, _I, _P, _P, _I, _P, _P, _P, _P], ctypes.c_int),
    "tacaw_build_potentials": ([_P, ctypes.POINTER(_Spec), _I, _I, _P, _P, _I,
                                ctypes.POINTER(ctypes.c_double), _P, _P, _P], ctypes.c_int),
    "tacaw_build_potentials_backward": ([_P, ctypes.POINTER(_Spec), _I, _I, _P, _P, _I,
                                         ctypes.POINTER(ctypes.c_double), _P, _P, _P], ctypes.c_int),
    "tacaw_multislice": ([_P, _I, ctypes.POINTER(_Job), _I, _I, _P], ctypes.c_int),
    "tacaw_multislice_adjoint": ([_P, _I, ctypes.POINTER(_Job), _I, ctypes.POINTER(_P),
                                  ctypes.POINTER(_P), _P], ctypes.c_int),
    "tacaw_periodogram": ([_P, _I, _I, _I, _I, _P, _I, _I, _P, _I, _P], ctypes.c_int),
    "tacaw_periodogram_positions": ([_P, _I, _I, _I, _I, _P, _I, _I, _I, _I, _P, _I, _P],
                                    ctypes.c_int),
    "tacaw_segstream_create": ([_P, _I, _I, _I, _I, _I, _P, ctypes.POINTER(_P)], ctypes.c_int),
    "tacaw_segstream_push": ([_P, _I, _P, _P], ctypes.c_int),
    "tacaw_segstream_finish": ([_P, ctypes.POINTER(_I), _P], ctypes.c_int),
    "tacaw_segstream_window": ([_P, ctypes.POINTER(_I), ctypes.POINTER(_I)], ctypes.c_int),
    "tacaw_segstream_destroy": ([_P], None),
    "tacaw_spectrum_finalize": ([_P, _I, _I, _P, ctypes.POINTER(_Opts), _P, _P, _P], ctypes.c_int),
    "tacaw_spectrum_finalize_noalloc": ([_P, _I, _I, _P, ctypes.POINTER(_Opts), _P, _P, _P],
                                        ctypes.c_int),
    "tacaw_autocorr_spectrum": ([_P, _I, _I, _I, _I, _P, ctypes.POINTER(_Opts), _P, _P, _P],
                                ctypes.c_int),
    "tacaw_autocorr_spectrum_backward": ([_P, _I, _I, _I, _I, _P, ctypes.POINTER(_Opts), _P, _P,
                                          _P, _P, _P], ctypes.c_int),
    "tacaw_energy_integrals": ([_P, _I, _I, _P, ctypes.POINTER(_Opts), _P, _P, _P], ctypes.c_int),
    "tacaw_qep_pattern": ([_P, _I, _I, _I, _I, _P, _I, _I, _I, _I, _I, _P, _P], ctypes.c_int),
    "tacaw_relative_difference": ([_P, _I, _I, _P, _P, _P, _P], ctypes.c_int),
    "tacaw_path_cut": ([_P, ctypes.c_double, ctypes.c_double, _I, _I, _I, _P, _I,
                        ctypes.POINTER(ctypes.c_double), _I, _P, _P], ctypes.c_int),
    "tacaw_autotune": ([_P, _I, _I, ctypes.c_char_p, _P], ctypes.c_int),
    "tacaw_load_tuning": ([_P, ctypes.c_char_p], ctypes.c_int),
    "tacaw_describe_schedule": ([_P, _I], ctypes.c_char_p),
    "tacaw_plan_count": ([_I], ctypes.c_int),
    "tacaw_set_timing": ([_P, _I], ctypes.c_int),
    "tacaw_set_potential_precision": ([_P, _I], ctypes.c_int),
    "tacaw_set_slice_blocking": ([_P, ctypes.c_int64, _I], ctypes.c_int),
    "tacaw_get_timing": ([_P, ctypes.c_char_p, ctypes.POINTER(KernelStats)], ctypes.c_int),
    "tacaw_set_cache_limits": ([_P, ctypes.c_int64, ctypes.c_int64, _I], ctypes.c_int),
    "tacaw_cache_stats": ([_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                           ctypes.POINTER(_I)], ctypes.c_int),
}
for _name, (_args, _res) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res

EXPORTED = tuple(_SIGS)


def _check(status):
    if status != 0:
        raise TacawError(f"tacaw status {status}: {_lib.tacaw_last_error().decode()}")


# ------------------------------------------------------------------------------------------------
# problem description

@dataclass
class Specimen:
    nx: int
    ny: int
    lx: float
    ly: float
    dz: Sequence[float]
    z0: float = 0.0
    bandlimit: float = 2.0 / 3.0

    def c(self):
        self._dz = np.ascontiguousarray(self.dz, dtype=np.float64)
        return _Spec(self.nx, self.ny, self.lx, self.ly, len(self._dz),
                     self._dz.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), self.z0,
                     self.bandlimit)

    @property
    def n_slices(self):
        return len(self.dz)


@dataclass
class Beam:
    energy_ev: float
    probe: bool = False
    alpha_rad: float = 0.0
    defocus_a: float = 0.0
    cs_a: float = 0.0
    probe_xy: Optional[np.ndarray] = None

    @property
    def n_pos(self):
        return 1 if not self.probe else int(np.asarray(self.probe_xy).shape[0])

    def c(self):
        if self.probe:
            self._pos = np.ascontiguousarray(self.probe_xy, dtype=np.float64).reshape(-1, 2)
            ptr = self._pos.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        else:
            ptr = None
        return _Beam(self.energy_ev, PROBE if self.probe else PLANE_WAVE, self.alpha_rad,
                     self.defocus_a, self.cs_a, self.n_pos, ptr)


@dataclass
class SpectrumOpts:
    dt_fs: float
    temperature_k: float
    n_e: int
    hop: int
    nqx_out: int
    nqy_out: int

    def c(self):
        return _Opts(self.dt_fs, self.temperature_k, self.n_e, self.hop, self.nqx_out, self.nqy_out)


def specimen_from(w):
    """Specimen from any object with nx, ny, lx, ly, dz, z0, bandlimit (e.g. a workloads.Workload)."""
    return Specimen(w.nx, w.ny, w.lx, w.ly, list(np.asarray(w.dz, dtype=np.float64)), w.z0,
                    w.bandlimit)


def beam_from(w):
    if w.probe:
        return Beam(w.energy_ev, True, w.alpha_rad, w.defocus_a, w.cs_a, np.asarray(w.probe_xy))
    return Beam(w.energy_ev)


# ------------------------------------------------------------------------------------------------
# context and stream plumbing

class Context:
    def __init__(self, device=0):
        h = _P()
        _check(_lib.tacaw_create(int(device), ctypes.byref(h)))
        self.handle = h
        self.device = device

    def __del__(self, _destroy=_lib.tacaw_destroy):
        # _destroy is bound at definition time: module globals may be gone at interpreter exit
        if getattr(self, "handle", None):
            _destroy(self.handle)
            self.handle = None


_ctx = {}


def context(device=0):
    """The process-wide context of a HIP device (created on first use)."""
    if device not in _ctx:
        _ctx[device] = Context(device)
    return _ctx[device]


def _stream(stream):
    if stream is not None:
        return _P(int(stream))
    import torch
    return _P(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise TacawError("expected a GPU tensor")
    if not t.is_contiguous():
        raise TacawError("expected a contiguous tensor")
    return _P(t.data_ptr())


def _dbl(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ------------------------------------------------------------------------------------------------
# entry points (same names as the C ABI)

def tacaw_version():
    return _lib.tacaw_version()


def tacaw_wavelength(energy_ev):
    return _lib.tacaw_wavelength(float(energy_ev))


def tacaw_interaction_parameter(energy_ev):
    return _lib.tacaw_interaction_parameter(float(energy_ev))


def tacaw_energy_axis(n_e, dt_fs):
    out = np.empty(n_e, dtype=np.float64)
    _check(_lib.tacaw_energy_axis(n_e, dt_fs, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out


def tacaw_bin_atoms(ctx, spec, xyz, species, n_species, offsets, order, n_outside=None, stream=None):
    s = spec.c()
    _check(_lib.tacaw_bin_atoms(ctx.handle, ctypes.byref(s), xyz.shape[0], xyz.shape[1], _ptr(xyz),
                                _ptr(species), n_species, _ptr(offsets), _ptr(order),
                                _ptr(n_outside), _stream(stream)))


def tacaw_build_potentials(ctx, spec, xyz, species, ff, V, n_outside=None, stream=None):
    s = spec.c()
    ffa, ffp = _dbl(ff)
    _check(_lib.tacaw_build_potentials(ctx.handle, ctypes.byref(s), xyz.shape[0], xyz.shape[1],
                                       _ptr(xyz), _ptr(species), ffa.shape[0], ffp, _ptr(V),
                                       _ptr(n_outside), _stream(stream)))


def tacaw_build_potentials_backward(ctx, spec, xyz, species, ff, grad_V, grad_xy, stream=None):
    s = spec.c()
    ffa, ffp = _dbl(ff)
    _check(_lib.tacaw_build_potentials_backward(ctx.handle, ctypes.byref(s), xyz.shape[0],
                                                xyz.shape[1], _ptr(xyz), _ptr(species),
                                                ffa.shape[0], ffp, _ptr(grad_V), _ptr(grad_xy),
                                                _stream(stream)))


@dataclass
class MsJob:
    spec: Specimen
    beam: Beam
    V: object                  # torch float32 [T][S][ny][nx] (cuda)
    exit: object               # torch complex64 [T][P][ny][nx] (cuda)
    ckpt: object = None        # torch complex64 [T][P][nck][ny][nx] (cuda) or None
    _keep: list = field(default_factory=list)


def _jobs(jobs):
    arr = (_Job * len(jobs))()
    keep = []
    for i, j in enumerate(jobs):
        s, b = j.spec.c(), j.beam.c()
        keep += [s, b]
        arr[i] = _Job(ctypes.pointer(s), ctypes.pointer(b), j.V.shape[0], _ptr(j.V),
                      _ptr(j.exit) if j.exit is not None else None, _ptr(j.ckpt))
    return arr, keep


def tacaw_multislice(ctx, jobs, ckpt_stride=0, mode=MODE_BATCHED, stream=None):
    arr, keep = _jobs(jobs)
    _check(_lib.tacaw_multislice(ctx.handle, len(jobs), arr, ckpt_stride, mode, _stream(stream)))


def tacaw_multislice_adjoint(ctx, jobs, ckpt_stride, grad_exit, grad_V, stream=None):
    arr, keep = _jobs(jobs)
    ge = (_P * len(jobs))(*[_ptr(g) for g in grad_exit])
    gv = (_P * len(jobs))(*[_ptr(g) for g in grad_V])
    _check(_lib.tacaw_multislice_adjoint(ctx.handle, len(jobs), arr, ckpt_stride, ge, gv,
                                         _stream(stream)))


def tacaw_periodogram(ctx, exit, n_e, hop, P_acc, accumulate=False, stream=None):
    T, Pn, ny, nx = exit.shape
    _check(_lib.tacaw_periodogram(ctx.handle, nx, ny, T, Pn, _ptr(exit), n_e, hop, _ptr(P_acc),
                                  1 if accumulate else 0, _stream(stream)))


def tacaw_periodogram_positions(ctx, exit, pos0, n_pos_used, n_e, hop, P_acc, accumulate=False,
                                stream=None):
    T, Pn, ny, nx = exit.shape
    _check(_lib.tacaw_periodogram_positions(ctx.handle, nx, ny, T, Pn, _ptr(exit), pos0, n_pos_used,
                                            n_e, hop, _ptr(P_acc), 1 if accumulate else 0,
                                            _stream(stream)))


class SegStream:
    """Streamed segment periodograms (tacaw_segstream_*): push exit-wave chunks [n][n_pos][ny][nx]
    in snapshot order, then finish() -> number of segments; P_acc then holds the periodogram."""

    def __init__(self, ctx, nx, ny, n_pos, n_e, hop, P_acc):
        h = _P()
        _check(_lib.tacaw_segstream_create(ctx.handle, nx, ny, n_pos, n_e, hop, _ptr(P_acc),
                                           ctypes.byref(h)))
        self.handle, self.P = h, P_acc

    def push(self, exit, stream=None):
        _check(_lib.tacaw_segstream_push(self.handle, exit.shape[0], _ptr(exit), _stream(stream)))

    def finish(self, stream=None):
        g = _I(0)
        _check(_lib.tacaw_segstream_finish(self.handle, ctypes.byref(g), _stream(stream)))
        return g.value

    def window(self):
        cap, held = _I(0), _I(0)
        _check(_lib.tacaw_segstream_window(self.handle, ctypes.byref(cap), ctypes.byref(held)))
        return cap.value, held.value

    def __del__(self, _destroy=_lib.tacaw_segstream_destroy):
        if getattr(self, "handle", None):
            _destroy(self.handle)
            self.handle = None


def tacaw_spectrum_finalize(ctx, P_acc, opts, S, norm=None, stream=None):
    _, ny, nx = P_acc.shape
    o = opts.c()
    _check(_lib.tacaw_spectrum_finalize(ctx.handle, nx, ny, _ptr(P_acc), ctypes.byref(o), _ptr(S),
                                        _ptr(norm), _stream(stream)))


def tacaw_spectrum_finalize_noalloc(ctx, P_acc, opts, S, norm=None, stream=None):
    _, ny, nx = P_acc.shape
    o = opts.c()
    _check(_lib.tacaw_spectrum_finalize_noalloc(ctx.handle, nx, ny, _ptr(P_acc), ctypes.byref(o),
                                                _ptr(S), _ptr(norm), _stream(stream)))


def tacaw_autocorr_spectrum(ctx, exit, opts, S, norm=None, stream=None):
    T, Pn, ny, nx = exit.shape
    o = opts.c()
    _check(_lib.tacaw_autocorr_spectrum(ctx.handle, nx, ny, T, Pn, _ptr(exit), ctypes.byref(o),
                                        _ptr(S), _ptr(norm), _stream(stream)))


def tacaw_autocorr_spectrum_backward(ctx, exit, opts, S, norm, grad_S, grad_exit, stream=None):
    T, Pn, ny, nx = exit.shape
    o = opts.c()
    _check(_lib.tacaw_autocorr_spectrum_backward(ctx.handle, nx, ny, T, Pn, _ptr(exit),
                                                 ctypes.byref(o), _ptr(S), _ptr(norm),
                                                 _ptr(grad_S), _ptr(grad_exit), _stream(stream)))


def tacaw_energy_integrals(ctx, P_acc, opts, c_tilde=None, c=None, stream=None):
    _, ny, nx = P_acc.shape
    o = opts.c()
    _check(_lib.tacaw_energy_integrals(ctx.handle, nx, ny, _ptr(P_acc), ctypes.byref(o),
                                       _ptr(c_tilde), _ptr(c), _stream(stream)))


def tacaw_qep_pattern(ctx, exit, t0, t_stride, t_count, out, stream=None):
    T, Pn, ny, nx = exit.shape
    nqy, nqx = out.shape
    _check(_lib.tacaw_qep_pattern(ctx.handle, nx, ny, T, Pn, _ptr(exit), t0, t_stride, t_count,
                                  nqx, nqy, _ptr(out), _stream(stream)))


def tacaw_relative_difference(ctx, A, B, out_row, stream=None):
    nqy, nqx = A.shape
    if tuple(B.shape) != (nqy, nqx) or out_row.numel() != nqx:
        raise TacawError("maps and profile must share the crop")
    _check(_lib.tacaw_relative_difference(ctx.handle, nqx, nqy, _ptr(A), _ptr(B), _ptr(out_row),
                                          _stream(stream)))


def tacaw_path_cut(ctx, lx, ly, S, vertices, n_per_seg, out, stream=None):
    n_e, nqy, nqx = S.shape
    arr, vp = _dbl(np.asarray(vertices, dtype=np.float64).reshape(-1, 2))
    n_vert = arr.shape[0]
    if out.shape[0] != n_e or out.shape[1] != (n_vert - 1) * n_per_seg + 1:
        raise TacawError("out must be [n_e][(n_vert - 1) * n_per_seg + 1]")
    _check(_lib.tacaw_path_cut(ctx.handle, float(lx), float(ly), nqx, nqy, n_e, _ptr(S), n_vert,
                               vp, n_per_seg, _ptr(out), _stream(stream)))


def tacaw_autotune(ctx, n, n_waves, cache_path=None, stream=None):
    _check(_lib.tacaw_autotune(ctx.handle, n, n_waves,
                               cache_path.encode() if cache_path else None, _stream(stream)))


def tacaw_load_tuning(ctx, cache_path):
    _check(_lib.tacaw_load_tuning(ctx.handle, cache_path.encode()))


def tacaw_plan_count(n):
    return int(_lib.tacaw_plan_count(n))


def tacaw_describe_schedule(ctx, n):
    return _lib.tacaw_describe_schedule(ctx.handle, n).decode()


def tacaw_set_potential_precision(ctx, split16):
    _check(_lib.tacaw_set_potential_precision(ctx.handle, int(split16)))


SLICE_BLOCK_BYTES = 192 << 20     # the library's defaults for tacaw_set_slice_blocking
SLICE_BLOCK_STREAMS = 2


def tacaw_set_slice_blocking(ctx, block_bytes, streams):
    _check(_lib.tacaw_set_slice_blocking(ctx.handle, int(block_bytes), int(streams)))


def tacaw_set_timing(ctx, enable):
    _check(_lib.tacaw_set_timing(ctx.handle, 1 if enable else 0))


def tacaw_get_timing(ctx, kind=None):
    st = KernelStats()
    _check(_lib.tacaw_get_timing(ctx.handle, kind.encode() if kind else None, ctypes.byref(st)))
    return dict(launches=st.launches, total_ms=st.total_ms, algo_bytes=st.algo_bytes)


def tacaw_set_cache_limits(ctx, max_entries, max_bytes, max_graphs):
    _check(_lib.tacaw_set_cache_limits(ctx.handle, int(max_entries), int(max_bytes), int(max_graphs)))


def tacaw_cache_stats(ctx):
    n, b, g = ctypes.c_int64(0), ctypes.c_int64(0), _I(0)
    _check(_lib.tacaw_cache_stats(ctx.handle, ctypes.byref(n), ctypes.byref(b), ctypes.byref(g)))
    return dict(tables=n.value, table_bytes=b.value, graphs=g.value)
