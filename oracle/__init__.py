"""FP64 CPU oracle of the RSM hot path — TEST INFRASTRUCTURE, not part of the product.

Only `tests/`, the smoke check in `__graft_entry__.py` and the CPU-baseline leg of
`bench.py` may import anything from here.  The HIP library never calls it, and nothing
here calls the HIP library: the two share no code.  The seeded input generators live
in their own package (`synth`) and hold none of the method's arithmetic.

Parity status of each function (what pins it, see tests/test_oracle_*.py):
  rng.philox4x64_10       known-answer test against numpy.random.Philox (library)
  rng.floyd_subsets       distinct / sorted / in range; chi-square uniformity over all
                          C(8,3) subsets
  rsm.qualifying_rows     brute force over rows and columns
  rsm.minor_right_...     noise-free: null on the true V rows of the chosen columns
                          (eq.(constrain.barV)); noisy: same projector as eigh(Z^T Z)
  rsm.accumulate_N        trace(N) = nvec * accepted; brute force over all C(n,l) subsets
                          for tiny n; noise-free N V-bar = 0
  rsm.solve_V             noise-free exact recovery (Theorem 1 with Psi = 0);
                          rho = 1, l = n gives the truncated SVD (Eckart-Young)
  rsm.solve_U             per-row lstsq; rho = 1 closed form U = Y V
  rsm.embed               eq.(get_xi) by hand; a shifted index also breaks the brute-force N
  rsm.error_e             the paper's printed Table I error at a Table I shape; the
                          definition eq.(ep) evaluated entry by entry
  metrics.principal_..    sine and cosine forms agree above 1e-8; a 1e-12 perturbation
                          is resolved by the sine form only
  metrics.rel_rms_known   the ratio summed entry by entry over the known entries only
                          (a dropped mask or the other normaliser fails it)
"""
from . import metrics, rng, rsm  # noqa: F401
from .rsm import OracleResult, rsm as run  # noqa: F401
