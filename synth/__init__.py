"""Seeded synthetic inputs shaped like the paper's workloads.

Shared by the tests, the benchmark and the oracle's callers.  Nothing here performs any
step of the decomposition method: it only draws matrices.

The model is the paper's synthetic generator, eq.(construct.Y) in Section V-A:
    Y-bar = randn(m, r) randn(r, n),  Psi = sigma randn(m, n),  W = rand(m, n) <= rho,
with W_ij = 1 marking a known entry (eq.(problem)).  Draw order is U, V, noise, mask,
from numpy's PCG64 seeded by `seed`; every matrix is filled in column-major order
(as Matlab fills randn(m, n)).

Layout of the returned arrays: `Yt` and `Wt` are C-contiguous (n, m) arrays, i.e. Y and
W stored column-major — the layout the device library reads without repacking.
`problem.Y` / `problem.W` give (m, n) views of the same memory.

Named workloads (the sizes every test and benchmark refers to):
  plain_fp64      2000 x 200, r=5, l=6, rho=0.7, noise N(0, 1e-3^2), 800 trials, FP64 end to end
  paper_scale     131072 x 1024, r=8, l=9, rho=0.8, FP32 factors, sigma = 1e-2 rms(UV^T),
                  8192 trials, Gram in FP32
  precision       131072 x 1024, r=8, rho=0.8, 16384 trials, Y = U diag(s) V^T with orthonormal
                  U, V and s geometric from 1 to 1e-3, noise 1e-5
  batched(k)      problem k of 256: m ~ U{4096..65536}, n ~ U{128..1024}, r ~ U{2..16},
                  rho ~ U[0.6, 0.9], l = r+1, 4n trials, FP32 factors, no noise term
  table1(row)     the paper's Table I shapes (r=3, l=4, I = 25 n)
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Problem:
    name: str
    m: int
    n: int
    r: int
    l: int
    num_submatrices: int
    seed_rsm: int
    rho: float
    gram: str                      # "f64" | "f32" | "bf16x2"
    Yt: np.ndarray                 # (n, m) C-contiguous == Y column-major
    Wt: np.ndarray                 # (n, m) uint8, 1 = known
    Ubar: np.ndarray | None = None  # ground-truth factors (None when not drawn)
    Vbar: np.ndarray | None = None  # n x r basis of the true row space
    sigma: float = 0.0
    meta: dict = field(default_factory=dict)

    @property
    def Y(self) -> np.ndarray:
        return self.Yt.T

    @property
    def W(self) -> np.ndarray:
        return self.Wt.T.view(bool) if self.Wt.dtype == np.uint8 else self.Wt.T


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(int(seed))))


def _randn_colmajor(rng, m, n, dtype=np.float64):
    """An m x n standard-normal matrix filled column by column, returned as (n, m) C-order."""
    return rng.standard_normal((n, m), dtype=dtype)


def _mask_colmajor(rng, m, n, rho):
    """W = rand(m, n) <= rho, filled column by column, returned as (n, m) uint8."""
    out = np.empty((n, m), dtype=np.uint8)
    step = max(1, (1 << 24) // max(1, m))
    for j0 in range(0, n, step):
        j1 = min(n, j0 + step)
        out[j0:j1] = rng.random((j1 - j0, m)) <= rho
    return out


def paper_synthetic(m, n, r, rho, sigma=0.0, seed=0, *, factor_dtype=np.float64,
                    y_dtype=np.float64, relative_sigma=False, num_submatrices=None,
                    l=None, seed_rsm=1, gram="f64", name="synthetic") -> Problem:
    """eq.(construct.Y): low-rank Gaussian factors plus iid Gaussian noise and an iid mask.

    factor_dtype: dtype the factors are drawn in (the product is formed in FP64 from them).
    relative_sigma: if True, the noise standard deviation is sigma * rms(U V^T).
    """
    rng = _rng(seed)
    Ubar = _randn_colmajor(rng, m, r).T.astype(factor_dtype).astype(np.float64)   # m x r
    Bt = _randn_colmajor(rng, r, n).T.astype(factor_dtype).astype(np.float64)     # (r, n) as randn(r, n)
    Yt = Bt.T @ Ubar.T                                                             # (n, m): Y-bar column-major
    noise_sd = float(sigma)
    if relative_sigma:
        noise_sd = float(sigma) * float(np.sqrt(np.mean(Yt * Yt)))
    if noise_sd > 0.0:
        Yt += noise_sd * _randn_colmajor(rng, m, n)
    Wt = _mask_colmajor(rng, m, n, rho)
    Yt = np.ascontiguousarray(Yt.astype(y_dtype))
    l = r + 1 if l is None else l
    I = 25 * n if num_submatrices is None else num_submatrices
    return Problem(name=name, m=m, n=n, r=r, l=l, num_submatrices=I, seed_rsm=seed_rsm,
                   rho=rho, gram=gram, Yt=Yt, Wt=Wt, Ubar=Ubar, Vbar=Bt.T.copy(),
                   sigma=noise_sd)


def spectrum_synthetic(m, n, r, rho, singular_values, noise, seed=0, *, y_dtype=np.float32,
                       num_submatrices=None, seed_rsm=1, gram="f32", name="precision") -> Problem:
    """Y = U diag(s) V^T + noise with orthonormal U, V (QR of Gaussian matrices, FP64)."""
    rng = _rng(seed)
    Ug, _ = np.linalg.qr(_randn_colmajor(rng, m, r).T)
    Vg, _ = np.linalg.qr(_randn_colmajor(rng, n, r).T)
    s = np.asarray(singular_values, dtype=np.float64)
    Yt = (Vg * s) @ Ug.T
    if noise > 0.0:
        Yt += noise * _randn_colmajor(rng, m, n)
    Wt = _mask_colmajor(rng, m, n, rho)
    Yt = np.ascontiguousarray(Yt.astype(y_dtype))
    return Problem(name=name, m=m, n=n, r=r, l=r + 1,
                   num_submatrices=(25 * n if num_submatrices is None else num_submatrices),
                   seed_rsm=seed_rsm, rho=rho, gram=gram, Yt=Yt, Wt=Wt, Ubar=Ug * s,
                   Vbar=Vg, sigma=float(noise), meta={"singular_values": s})


# ---------------------------------------------------------------- named workloads

def plain_fp64(seed: int = 0, seed_rsm: int = 1) -> Problem:
    return paper_synthetic(2000, 200, 5, 0.7, 1e-3, seed, num_submatrices=800, l=6,
                           seed_rsm=seed_rsm, gram="f64", name="plain_fp64 2000x200 r5")


def paper_scale(seed: int = 0, seed_rsm: int = 1, m: int = 131072, n: int = 1024,
                num_submatrices: int = 8192) -> Problem:
    return paper_synthetic(m, n, 8, 0.8, 1e-2, seed, factor_dtype=np.float32,
                           y_dtype=np.float32, relative_sigma=True,
                           num_submatrices=num_submatrices, l=9, seed_rsm=seed_rsm,
                           gram="f32", name=f"paper_scale {m}x{n} r8")


def precision_stress(seed: int = 0, seed_rsm: int = 1, m: int = 131072, n: int = 1024,
                     num_submatrices: int = 16384, gram: str = "f32") -> Problem:
    s = 10.0 ** (-3.0 * np.arange(8) / 7.0)
    return spectrum_synthetic(m, n, 8, 0.8, s, 1e-5, seed, num_submatrices=num_submatrices,
                              seed_rsm=seed_rsm, gram=gram, name=f"precision {m}x{n} r8")


def batched_sizes(count: int = 256, seed: int = 3) -> list[dict]:
    """Sizes of the mixed batch: m ~ U{4096..65536}, n ~ U{128..1024}, r ~ U{2..16},
    rho ~ U[0.6, 0.9], l = r+1, 4n trials; one data seed and one RSM seed per problem."""
    rng = _rng(seed)
    m = rng.integers(4096, 65536, size=count, endpoint=True)
    n = rng.integers(128, 1024, size=count, endpoint=True)
    r = rng.integers(2, 16, size=count, endpoint=True)
    rho = rng.uniform(0.6, 0.9, size=count)
    data_seeds = rng.integers(0, 2**31 - 1, size=count)
    rsm_seeds = rng.integers(0, 2**62, size=count)
    return [dict(m=int(m[k]), n=int(n[k]), r=int(r[k]), l=int(r[k]) + 1, rho=float(rho[k]),
                 num_submatrices=4 * int(n[k]), seed=int(data_seeds[k]),
                 seed_rsm=int(rsm_seeds[k])) for k in range(count)]


def batched_problem(spec: dict, gram: str = "f32") -> Problem:
    return paper_synthetic(spec["m"], spec["n"], spec["r"], spec["rho"], 0.0, spec["seed"],
                           factor_dtype=np.float32, y_dtype=np.float32,
                           num_submatrices=spec["num_submatrices"], l=spec["l"],
                           seed_rsm=spec["seed_rsm"], gram=gram,
                           name=f"batched {spec['m']}x{spec['n']} r{spec['r']}")


def batched_device(spec: dict, device="cuda"):
    """The same recipe drawn on the device (torch's generator seeded with spec["seed"]):
    U (m x r), V (n x r) iid N(0,1) in FP32, Y = fl32(U V^T) formed in FP64, W iid
    Bernoulli(rho).  Returns (Y, W) as column-major (m, n) views.  For workloads too large
    to draw on the host in seconds; the values differ from batched_problem's."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(spec["seed"]))
    m, n, r, rho = spec["m"], spec["n"], spec["r"], spec["rho"]
    U = torch.randn(m, r, generator=g, device=device, dtype=torch.float32)
    V = torch.randn(n, r, generator=g, device=device, dtype=torch.float32)
    Yt = (V.double() @ U.double().T).float()                 # (n, m): Y column-major
    Wt = torch.rand(n, m, generator=g, device=device) < rho
    return Yt.T, Wt.T


# The paper's Table I rows: (m, n, rho, sigma); r = 3, l = 4 (Section V-A).
TABLE1_ROWS = [
    (65536, 1024, 0.2, 0.2), (98304, 1024, 0.2, 0.2), (131072, 1024, 0.2, 0.2),
    (131072, 768, 0.2, 0.2), (131072, 512, 0.2, 0.2), (131072, 1024, 0.5, 0.1),
    (131072, 1024, 0.4, 0.1), (131072, 1024, 0.3, 0.1), (131072, 1024, 0.3, 0.3),
    (131072, 1024, 0.3, 0.5),
]


def table1(row: int, seed: int = 0, seed_rsm: int = 1, trials_per_column: int = 25) -> Problem:
    m, n, rho, sigma = TABLE1_ROWS[row]
    return paper_synthetic(m, n, 3, rho, sigma, seed, num_submatrices=trials_per_column * n,
                           l=4, seed_rsm=seed_rsm, gram="f64", name=f"table1[{row}] {m}x{n}")
