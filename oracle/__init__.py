"""FP64 CPU oracle for gradient projection with adaptive steplengths (GPSS).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import anything from this package; the
product library never calls it, and this package imports nothing from the
product (it shares no kernels, helpers, tables or constants with it).

Everything is plain numpy in float64, written from the paper
(Loris, Bertero, De Mol, Zanella, Zanni, "Accelerating gradient projection
methods for l1-constrained signal recovery by steplength selection rules"):

  * projection.py - Euclidean projection onto the l1 ball (sort based).
  * gpss.py       - Algorithm 1 (gradient projection) driven by Algorithm 2
                    (adaptive Barzilai-Borwein alternation), Section 3.
  * fom.py        - the comparison methods of Section 2: ISTA (item 1),
                    FISTA (item 2, equation (3)) and projected steepest
                    descent (item 5).
  * lista.py      - unrolled soft-thresholding network (ISTA of Section 2,
                    item 1, with learned matrices) forward and backward pass.
  * exact.py      - exact references used to pin the above: brute-force
                    enumeration of the constrained least-squares solution and
                    the lambda <-> rho relation of Section 1.
"""
from .projection import project_l1, project_l1_mu, soft_threshold
from .gpss import GPSSParams, gpss, ss_update, STATUS_NAMES

__all__ = ["project_l1", "project_l1_mu", "soft_threshold", "GPSSParams",
           "gpss", "ss_update", "STATUS_NAMES"]
