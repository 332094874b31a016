"""Counter-based pseudo-random numbers (SplitMix64, Steele, Lea & Flood 2014).

Value ``i`` of stream ``seed`` is the SplitMix64 finaliser applied to
``seed + (i + 1) * 0x9E3779B97F4A7C15 (mod 2**64)``.  Because every value is a
pure function of ``(seed, i)`` the same numbers come out on the CPU and on the
GPU, in any chunking.  Arithmetic is done in torch int64, whose multiplication
wraps modulo 2**64 like uint64; right shifts are made logical with a mask.
"""
import math

import torch

_GOLDEN = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB


def _s64(c):
    """Reinterpret a uint64 constant as the int64 with the same bits."""
    return c - (1 << 64) if c >= (1 << 63) else c


def _lsr(z, k):
    """Logical right shift of int64 bits."""
    return (z >> k) & ((1 << (64 - k)) - 1)


def splitmix64_u64(seed, count, offset=0, device="cpu"):
    """Raw 64-bit outputs (as int64 bit patterns) of stream ``seed``, indices offset..offset+count-1."""
    idx = torch.arange(offset + 1, offset + count + 1, dtype=torch.int64, device=device)
    z = idx * _s64(_GOLDEN) + _s64(seed % (1 << 64))
    z = (z ^ _lsr(z, 30)) * _s64(_M1)
    z = (z ^ _lsr(z, 27)) * _s64(_M2)
    return z ^ _lsr(z, 31)


def uniform01(seed, shape, device="cpu", offset=0):
    """Doubles in [0, 1): the top 53 bits of each SplitMix64 output times 2**-53."""
    n = math.prod(shape)
    z = splitmix64_u64(seed, n, offset=offset, device=device)
    return (_lsr(z, 11).to(torch.float64) * (2.0 ** -53)).reshape(shape)


def uniform_pm1(seed, shape, device="cpu", offset=0):
    """Doubles in [-1, 1)."""
    return 2.0 * uniform01(seed, shape, device=device, offset=offset) - 1.0


def gaussian(seed, shape, device="cpu"):
    """Standard normal doubles by Box-Muller on consecutive uniform pairs (u1, u2).

    u1 is mapped to (0, 1] so the logarithm is finite.
    """
    n = math.prod(shape)
    m = (n + 1) // 2
    u = uniform01(seed, (m, 2), device=device)
    r = torch.sqrt(-2.0 * torch.log1p(-u[:, 0]))
    t = 2.0 * math.pi * u[:, 1]
    out = torch.stack((r * torch.cos(t), r * torch.sin(t)), dim=1).reshape(-1)[:n]
    return out.reshape(shape)
