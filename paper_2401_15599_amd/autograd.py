"""torch.autograd.Functions over the library's forward and adjoint entry points.

TacawPotentials: positions [T][N][3] -> V [T][S][ny][nx]         (backward: dL/d(x, y); dL/dz = 0)
TacawMultislice: V -> exit waves [T][P][ny][nx] complex64        (backward: checkpointed adjoint)
TacawSpectrum:   exit waves -> I(q, E) [n_e][nqy][nqx]            (backward: spectrum adjoint)

Each forward and backward is a single call into libtacaw; tensors stay on the GPU and the work
runs on torch's current stream.  Complex gradients follow torch's convention
(dL/dRe + i dL/dIm), which is the convention of the C ABI.
"""
import math

import torch

from . import (MsJob, context, tacaw_autocorr_spectrum, tacaw_autocorr_spectrum_backward,
               tacaw_build_potentials, tacaw_build_potentials_backward, tacaw_multislice,
               tacaw_multislice_adjoint, MODE_BATCHED)


class TacawPotentials(torch.autograd.Function):
    @staticmethod
    def forward(ctx, xyz, species, spec, ff):
        ctx_ = context(xyz.device.index or 0)
        T = xyz.shape[0]
        V = torch.empty((T, spec.n_slices, spec.ny, spec.nx), dtype=torch.float32, device=xyz.device)
        xyz = xyz.contiguous()
        species = species.contiguous()
        tacaw_build_potentials(ctx_, spec, xyz, species, ff, V)
        ctx.save_for_backward(xyz, species)
        ctx.spec, ctx.ff = spec, ff
        return V

    @staticmethod
    def backward(ctx, gV):
        xyz, species = ctx.saved_tensors
        gxy = torch.empty((xyz.shape[0], xyz.shape[1], 2), dtype=torch.float32, device=xyz.device)
        tacaw_build_potentials_backward(context(xyz.device.index or 0), ctx.spec, xyz, species,
                                        ctx.ff, gV.contiguous(), gxy)
        g = torch.zeros_like(xyz)
        g[..., :2] = gxy
        return g, None, None, None


class TacawMultislice(torch.autograd.Function):
    @staticmethod
    def forward(ctx, V, spec, beam, ckpt_stride):
        T = V.shape[0]
        P = beam.n_pos
        k = ckpt_stride if ckpt_stride else max(1, math.ceil(math.sqrt(spec.n_slices)))
        nck = (spec.n_slices + k - 1) // k
        exit = torch.empty((T, P, spec.ny, spec.nx), dtype=torch.complex64, device=V.device)
        ckpt = torch.empty((T, P, nck, spec.ny, spec.nx), dtype=torch.complex64, device=V.device)
        V = V.contiguous()
        tacaw_multislice(context(V.device.index or 0), [MsJob(spec, beam, V, exit, ckpt)],
                         ckpt_stride=k, mode=MODE_BATCHED)
        ctx.save_for_backward(V, ckpt)
        ctx.spec, ctx.beam, ctx.k = spec, beam, k
        return exit

    @staticmethod
    def backward(ctx, gexit):
        V, ckpt = ctx.saved_tensors
        gV = torch.empty_like(V)
        tacaw_multislice_adjoint(context(V.device.index or 0),
                                 [MsJob(ctx.spec, ctx.beam, V, None, ckpt)], ctx.k,
                                 [gexit.contiguous()], [gV])
        return gV, None, None, None


class TacawSpectrum(torch.autograd.Function):
    @staticmethod
    def forward(ctx, exit, opts):
        S = torch.empty((opts.n_e, opts.nqy_out, opts.nqx_out), dtype=torch.float32,
                        device=exit.device)
        norm = torch.empty((1,), dtype=torch.float64, device=exit.device)
        exit = exit.contiguous()
        tacaw_autocorr_spectrum(context(exit.device.index or 0), exit, opts, S, norm)
        ctx.save_for_backward(exit, S, norm)
        ctx.opts = opts
        return S

    @staticmethod
    def backward(ctx, gS):
        exit, S, norm = ctx.saved_tensors
        gexit = torch.empty_like(exit)
        tacaw_autocorr_spectrum_backward(context(exit.device.index or 0), exit, ctx.opts, S, norm,
                                         gS.contiguous(), gexit)
        return gexit, None
