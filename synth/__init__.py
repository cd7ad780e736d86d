"""Seeded synthetic F-engine output for the 4-bit X-engine.

This module holds no correlation arithmetic. It only draws inputs, so both the
GPU path's tests and the CPU oracle's tests can be fed the same bytes.

Recipe (the paper's data are CHIME F-engine samples, which are not available
here): each complex sample's real and imaginary parts are drawn independently
as sigma * N(0, 1), rounded to the nearest integer (ties to even), clipped to
[-8, 7] and stored Excess-8 (value + 8) in one byte, real part in the high
nibble (paper Sec. III: 4+4-bit offset-encoded complex samples; the nibble order
is this library's stated reading). A common complex component of amplitude
``common`` shared by all elements of one (channel, time) can be mixed in before
quantisation, which gives the matrix non-trivial off-diagonal structure like a
bright source on the sky.
"""
from __future__ import annotations

import numpy as np
import torch

VALUE_MIN = -8
VALUE_MAX = 7


def pack(q_re, q_im):
    """Excess-8 byte from signed parts in [-8, 7]: ((re + 8) << 4) | (im + 8)."""
    q_re = np.asarray(q_re, dtype=np.int16)
    q_im = np.asarray(q_im, dtype=np.int16)
    if q_re.size and (q_re.min() < VALUE_MIN or q_re.max() > VALUE_MAX
                      or q_im.min() < VALUE_MIN or q_im.max() > VALUE_MAX):
        raise ValueError("4-bit values must lie in [-8, 7]")
    return (((q_re + 8) << 4) | (q_im + 8)).astype(np.uint8)


def _pack_torch(q_re: torch.Tensor, q_im: torch.Tensor) -> torch.Tensor:
    return (((q_re + 8) << 4) | (q_im + 8)).to(torch.uint8)


def _quantise(z: torch.Tensor) -> torch.Tensor:
    return torch.clamp(torch.round(z), VALUE_MIN, VALUE_MAX).to(torch.int16)


def quantized_gaussian(f: int, t: int, n: int, sigma: float, seed: int, common: float = 0.0,
                       device="cpu", return_parts: bool = False):
    """uint8[F][T][N] packed samples (torch tensor on ``device``).

    Drawn channel block by channel block from one torch generator seeded with
    ``seed``, so the bytes depend only on (shape, sigma, common, seed, device
    type). With ``return_parts`` the signed parts (int16) come back as well.
    """
    device = torch.device(device)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    out = torch.empty((f, t, n), dtype=torch.uint8, device=device)
    parts_re = parts_im = None
    if return_parts:
        parts_re = torch.empty((f, t, n), dtype=torch.int16, device=device)
        parts_im = torch.empty((f, t, n), dtype=torch.int16, device=device)
    per = max(1, (1 << 26) // max(1, t * n))        # ~64M samples per block
    for f0 in range(0, f, per):
        fc = min(per, f - f0)
        zr = torch.randn((fc, t, n), generator=gen, device=device)
        zi = torch.randn((fc, t, n), generator=gen, device=device)
        if common:
            sr = torch.randn((fc, t, 1), generator=gen, device=device)
            si = torch.randn((fc, t, 1), generator=gen, device=device)
            zr += common * sr
            zi += common * si
        qr = _quantise(zr * sigma)
        qi = _quantise(zi * sigma)
        out[f0:f0 + fc] = _pack_torch(qr, qi)
        if return_parts:
            parts_re[f0:f0 + fc] = qr
            parts_im[f0:f0 + fc] = qi
        del zr, zi
    if return_parts:
        return out, parts_re, parts_im
    return out


def uniform_bytes(f: int, t: int, n: int, seed: int, device="cpu") -> torch.Tensor:
    """Every byte value equally likely (exercises the full [-8, 7] range)."""
    gen = torch.Generator(device=torch.device(device))
    gen.manual_seed(int(seed))
    return torch.randint(0, 256, (f, t, n), generator=gen, dtype=torch.uint8, device=device)


def constant_bytes(f: int, t: int, n: int, value: int, device="cpu") -> torch.Tensor:
    return torch.full((f, t, n), int(value), dtype=torch.uint8, device=device)
