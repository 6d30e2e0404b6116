"""Counter-based random numbers for the synthetic inputs.

Every random value is a pure function of (seed, field id, linear index), so
any sub-block of a field can be generated on its own (CPU or GPU, in chunks)
and reproduce the same numbers bit for bit.

    u = (splitmix64(splitmix64(seed) ^ (field << 56) ^ index) >> 11) * 2**-53

splitmix64 is Steele, Lea & Flood, "Fast splittable pseudorandom number
generators" (OOPSLA 2014), with the constants published there.  Torch int64
arithmetic wraps modulo 2**64; logical right shifts are emulated with masks.
"""
import torch

_GOLDEN = 0x9E3779B97F4A7C15
_MIX1 = 0xBF58476D1CE4E5B9
_MIX2 = 0x94D049BB133111EB
_M64 = (1 << 64) - 1


def _signed(c):
    c &= _M64
    return c - (1 << 64) if c >= (1 << 63) else c


def _lsr(z, s):
    """Logical right shift of an int64 tensor."""
    return (z >> s) & ((1 << (64 - s)) - 1)


def splitmix64_int(x):
    """Reference splitmix64 on a Python int (unsigned 64-bit)."""
    z = (x + _GOLDEN) & _M64
    z = ((z ^ (z >> 30)) * _MIX1) & _M64
    z = ((z ^ (z >> 27)) * _MIX2) & _M64
    return z ^ (z >> 31)


def splitmix64(x):
    """splitmix64 on an int64 tensor (values read as unsigned 64-bit)."""
    z = x + _signed(_GOLDEN)
    z = (z ^ _lsr(z, 30)) * _signed(_MIX1)
    z = (z ^ _lsr(z, 27)) * _signed(_MIX2)
    return z ^ _lsr(z, 31)


def uniform(seed, field, index):
    """U[0,1) doubles for an int64 tensor of linear indices."""
    key = splitmix64_int(seed & _M64) ^ ((field & 0xFF) << 56)
    z = splitmix64(index ^ _signed(key))
    return _lsr(z, 11).to(torch.float64) * (2.0 ** -53)


def symmetric(seed, field, index):
    """U[-1,1) doubles."""
    return 2.0 * uniform(seed, field, index) - 1.0


def gaussian(seed, field, index):
    """Standard normal doubles by Box-Muller from two counter streams."""
    u1 = uniform(seed, field, 2 * index)
    u2 = uniform(seed, field, 2 * index + 1)
    r = torch.sqrt(-2.0 * torch.log1p(-u1))
    return r * torch.cos(2.0 * torch.pi * u2)
