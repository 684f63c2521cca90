"""FP64 CPU oracle for the per-band HRMS reconstruction under the local Laplacian prior (LLP).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's CPU-baseline leg import this
package; the library's product path never does, and nothing here is shared with the HIP implementation.

Every function states the passage of the paper it follows.  Pins (checks against brute force, closed forms and
identities that do not reuse this code) live in the CPU test suite.  Functions without such a pin say
"parity unpinned" in their docstring.
"""
from .llp import (  # noqa: F401
    Problem,
    apply_A,
    apply_data,
    apply_llp,
    blur,
    blur_adjoint,
    cg,
    decimate,
    decimate_adjoint,
    kernel_otf,
    laplacian,
    laplacian_symbol,
    matting_apply,
    matting_diag_mean,
    matting_stats,
    objective,
    objective_levin,
    pcg,
    precond_apply,
    rhs,
    solve,
    window_sum,
)
from . import polish  # noqa: F401,E402  (the A, C step and the Z step of Algorithm "Fast Pansharpening")
from . import tgv  # noqa: F401,E402  (Algorithm "Blur Kernel Estimation", host side)
from . import lgc  # noqa: F401,E402  (the LGC prior of eq. reg2_lgc, the comparison prior)
from . import priors  # noqa: F401,E402  (the filter priors of the cross-channel prior comparison)
