"""MI355X-native differentiable forward model of PMF-STGR (arXiv 2503.22139).

The five steps of the Stage 2/3 training iteration (Sec. 2.3.2): voxelize the
reference-frame Gaussians (Eq. 5), voxelize the signed motion-basis Gaussians,
combine the bases with per-projection coefficients into DVFs (Eq. 3), warp the
reference volume (Eq. 2) and cone-beam project each warped volume (Eq. 6),
each with its adjoint.  The compute runs in the HIP library ``libpmf.so``
(C ABI declared in ``include/pmf.h``); ``ops`` is its Python binding.

Importing the package loads nothing: ``synth`` (input generators) works on a
machine without a GPU, and ``ops`` loads the library on first use and raises
if it is missing.
"""

__all__ = ["synth", "ops"]
__version__ = "0.1.0"
