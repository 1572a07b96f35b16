"""MI355X (gfx950) implementation of the coupled FD-LBM step for catalytic
reactive flow (Kulyk, Berger, Smith, Harting).  The method runs in the HIP
library libfdlbm.so (C ABI in include/fdlbm.h); `fdlbm.Sim` is its binding
and `workloads` generates seeded synthetic inputs."""
from . import workloads  # noqa: F401
