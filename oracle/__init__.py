"""FP64 CPU oracle for the LoopSplat rendering/registration hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) imports, calls or links this package; only the test-suite, the
smoke check and the CPU-baseline leg of the benchmark do.  It shares no code
with the GPU path: it is written from the mathematics of the paper and of EWA
splatting, in plain float64 PyTorch CPU ops (gradients by autograd of the
forward written here), NumPy and pure-Python loops for small cases.

Modules
  raster    projection (EWA), tile binning, front-to-back compositing, L1 loss
  register  Adam, per-view keyframe localisation, weighted rotation averaging
            (paper Sec. 3.2, Eq. 7), transform errors
  mapping   submap-update loss: L1 + SSIM colour term, depth term and the
            isotropic scale regulariser (paper Sec. 3.1, Eq. 3-5)
  adjust    rigid map adjustment of submaps and keyframe poses after pose-graph
            optimisation (paper Sec. 3.3, Eq. 8)
  overlap   geometric overlap ratio of two submaps by reciprocal nearest
            neighbours (supplement, loop detection, Eq. 9)
  prune     opacity pruning of a submap after mapping (supplement, submap
            update)

Every function with no independent pin is marked "parity unpinned" in its
docstring; the pins live in tests/test_oracle_*.py.
"""

from . import adjust, mapping, overlap, prune, raster, register  # noqa: F401
