"""MI355X-native QVA state-evolution engine (QAOA / QWOA hot path).

The computation lives in libqva.so (HIP, gfx950), reached through the C ABI
of include/qva.h; this package is a thin binding that passes PyTorch device
memory and streams to it.
"""

from ._lib import QvaError, load as load_library  # noqa: F401
from .qva import (  # noqa: F401
    Batch,
    Problem,
    QVAExpectation,
    evolve,
    evolve_noalloc,
    expectation,
    expectation_value,
    grad,
    init_uniform,
    mix_circulant,
    mix_x,
    parity_ring_pairs,
    phase,
)

__version__ = "0.1.0"
