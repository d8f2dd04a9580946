"""Seeded synthetic CP problems generated on the GPU with torch.

The same recipe as `cpgen.synth` (collinear factors A = sqrt(I) Q L^T with
L L^T = (1-c) I + c 11^T, the CP tensor of the truth, Gaussian noise at a
given SNR, independent N(0,1) starting factors).  It is used for request
pools too large to build on the host; the shape and parameter draws come from
a NumPy PCG64 stream, the tensor entries from a seeded torch generator on the
device.  Real problems are stored FP32, complex ones complex64 (real and
imaginary parts N(0,1)/sqrt(2), as for the host generator).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class DeviceProblem:
    dims: tuple
    R: int
    complex_: bool
    y: "object"          # 1-D torch tensor on the device, vec(Y) first index fastest
    init: list           # numpy (I_n, R) starting factors (float64 / complex128)
    c: float
    snr_db: float


def _randn(torch, shape, gen, complex_, dtype_real):
    if complex_:
        re = torch.randn(shape, generator=gen, device="cuda", dtype=dtype_real)
        im = torch.randn(shape, generator=gen, device="cuda", dtype=dtype_real)
        return torch.complex(re, im) / math.sqrt(2.0)
    return torch.randn(shape, generator=gen, device="cuda", dtype=dtype_real)


def _collinear(torch, I, R, c, gen, complex_):
    G = _randn(torch, (I, R), gen, complex_, torch.float64)
    if I >= R:
        Q, _ = torch.linalg.qr(G)
    else:
        Q = G / math.sqrt(I)
    S = (1.0 - c) * np.eye(R) + c * np.ones((R, R))
    L = torch.from_numpy(np.linalg.cholesky(S)).to(device="cuda", dtype=Q.dtype)
    return math.sqrt(I) * (Q @ L.T)


def cp_tensor_device(torch, factors):
    """vec of sum_r a_r^(1) o ... o a_r^(N) via the mode-1 unfolding (first index fastest)."""
    kr = factors[1]
    for A in factors[2:]:
        # Khatri-Rao with the earlier mode varying fastest: kr[(i1 + I1 i2), r]
        kr = (A[:, None, :] * kr[None, :, :]).reshape(-1, kr.shape[1])
    Y1 = factors[0] @ kr.T          # I_1 x prod_{k>1} I_k
    return Y1.T.contiguous().reshape(-1)  # column-major vec


def make_pool(torch, seed: int, count: int, n_choices=(3, 4), imin=16, imax=256, rmin=2, rmax=20,
              complex_frac=0.2, snr_db=20.0, max_elems=1 << 30):
    """`count` problems: N uniform over n_choices, I_n log-uniform in [imin, imax]
    (rounded), R ~ U{rmin..rmax}, c ~ U[0, 0.95], complex with probability
    complex_frac.  Shapes whose element count exceeds max_elems are redrawn."""
    rng = np.random.default_rng(seed)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    out = []
    while len(out) < count:
        N = int(rng.choice(n_choices))
        dims = tuple(int(round(math.exp(rng.uniform(math.log(imin), math.log(imax))))) for _ in range(N))
        R = int(rng.integers(rmin, rmax + 1))
        c = float(rng.uniform(0.0, 0.95))
        cplx = bool(rng.random() < complex_frac)
        if int(np.prod(dims)) > max_elems:
            continue
        truth = [_collinear(torch, I, R, c, gen, cplx) for I in dims]
        y = cp_tensor_device(torch, truth)
        J = y.numel()
        sigma = 10.0 ** (-snr_db / 20.0) * torch.linalg.vector_norm(y).item() / math.sqrt(J)
        y = y + sigma * _randn(torch, (J,), gen, cplx, torch.float64)
        y = y.to(torch.complex64 if cplx else torch.float32).contiguous()
        init = []
        for I in dims:
            if cplx:
                A = (rng.standard_normal((I, R)) + 1j * rng.standard_normal((I, R))) / np.sqrt(2.0)
            else:
                A = rng.standard_normal((I, R))
            init.append(np.asfortranarray(A))
        out.append(DeviceProblem(dims, R, cplx, y, init, c, snr_db))
        del truth
    return out
