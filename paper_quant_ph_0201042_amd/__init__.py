"""MI355X (gfx950) state-vector gate engine of the Niwa-Matsumoto-Imai
simulator: dense 2^n complex registers in HBM evolved by one-qubit and
controlled one-qubit gates in hand-written HIP kernels (libsv.so, C ABI in
include/sv.h).  PyTorch supplies device memory and streams."""

from ._lib import SVError, load as load_library  # noqa: F401
from .state import (  # noqa: F401
    State,
    adjoint,
    config_get,
    config_set,
    gate_dmatrix,
    gate_matrix,
    overlap_loss,
    jit_source,
    model_fused,
    plan_blocks,
    plan_fused,
)
from .autograd import OverlapLoss, overlap_loss_fn  # noqa: F401
from .batch import Batch, trajectory_gates  # noqa: F401
from . import autotune, experiments, shor  # noqa: F401,E402

load_library()
