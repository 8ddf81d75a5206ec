"""MI355X-native Fast Finite Shearlet Transform (FFST).

The transform of Haeuser & Steidl, "Fast Finite Shearlet Transform: a
tutorial": forward c_i = ifft2(Psi_i * fft2(f)) for every shearlet spectrum
Psi_i (eq. shearletTransform), adjoint / inverse
f = ifft2(sum_i Psi_i * fft2(c_i)) (eq. inverseShearletTransform), computed
by hand-written HIP kernels for gfx950 behind the C ABI of include/ffst.h.

    import torch
    from paper_1202_1773_amd import Plan
    plan = Plan(512, 512, J=3)                 # spectra generated on the GPU
    c = plan.forward(x)                        # x: (B, 512, 512) float32 cuda
    y = plan.adjoint(c)                        # (B, 512, 512)

    from paper_1202_1773_amd import BatchPlan  # images of several sizes
    bp = BatchPlan([(256, 256), (384, 512), (1024, 1024)])
    coeffs = bp.forward(bp.pack(images))       # one HIP graph launch

PyTorch supplies device memory and the current stream only.
"""

from ._lib import FfstError  # noqa: F401
from .batch import BatchPlan  # noqa: F401
from .plan import Plan  # noqa: F401
