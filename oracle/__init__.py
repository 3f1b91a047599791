"""Plain FP64 CPU oracle of regularized inverse holographic volume reconstruction.

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this package.  It shares no code with the GPU
library (no kernels, headers, tables or helpers) and never calls it.

Modules:
  optics  - angular-spectrum forward model A, its adjoint, ||A||^2 closed form
  prox    - 3D TV, gradient-projection TV prox, soft threshold, fused-lasso prox
  fista   - objective and the FISTA iteration
  detect  - threshold / connected components / weighted centroids / matching
  unet    - warm-start 3D U-Net forward and analytic backward
  complex_object - the complex-valued object: forward, adjoint, complex TV
            prox, complex shrinkage, objective and FISTA
"""
from . import optics, prox, fista, detect  # noqa: F401
from . import complex_object  # noqa: F401,E402
from . import unet  # noqa: F401,E402
