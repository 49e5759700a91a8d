"""MI355X explicit divergence-free DG (hot path of the method as a HIP library + binding)."""
from .dfdg import (  # noqa: F401
    Solver,
    Mesh,
    DfdgError,
    load_library,
    LIB_PATH,
    EXPORTED,
)
