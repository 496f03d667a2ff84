"""FP64 CPU oracle for black-box randomized HBS compression (Levitt & Martinsson,
"Linear-complexity black-box randomized compression of rank-structured
matrices", arXiv 2205.02990).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, literal NumPy/SciPy
(LAPACK) transcription of what the paper defines, one box at a time, written to
be checked by eye against the paper.  Only the test suite, the smoke check and
the CPU-baseline leg of the benchmark may import it; the product library never
does, and it shares no code with the GPU path (inputs come from the separate
``inputs`` module, which holds no arithmetic of the method).

Modules
  tree      cluster tree of section 3.1
  linalg    QR, col, null and the pseudo-inverse of sections 2.2-2.4 and 4.2
  hbs       compression (Algorithm 2), apply (Algorithm 1), dense telescoping
            reconstruction (section 3.3)
  logkernel the log-kernel stand-in black box (dense rows and samples)
  metrics   relative apply error on probes and the power-iteration norm
            estimate of section 5
"""
from . import tree, linalg, hbs, logkernel, metrics  # noqa: F401
