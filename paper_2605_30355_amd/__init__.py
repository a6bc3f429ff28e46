"""MI355X (gfx950) implementation of the Cosm sweep: a thin Python binding over
the C ABI of ``libcosm.so`` (declared in ``include/cosm.h``).

Every step of the method runs in the library's HIP kernels; this package only
marshals arguments.  PyTorch supplies device memory (the state's workspace)
and the HIP stream.  Importing the package does not touch the GPU; creating a
``State`` does, and fails loudly when the library has not been built.
"""
from .cosm import (  # noqa: F401
    COLOR_BALANCED, COLOR_GREEDY, COLOR_MINIMUM, COLOR_MISRA_GRIES, COLOR_TORUS,
    LDS_FORM_AUTO, LDS_FORM_PAIR, LDS_FORM_REGISTER, LDS_FORM_REGISTER_STREAM,
    ORDER_LARGEST_LAST,
    RES_AUTO, RES_HBM, RES_LDS, RES_PLAIN,
    READOUT_BISECTORS, READOUT_OPTIMAL,
    SCHED_CONTINUOUS, SCHED_GRID,
    STORE_BF16, STORE_FIX16, STORE_FIX32, STORE_FP16, STORE_FP16_PK, STORE_FP32,
    UNIT_DEGREES, UNIT_RADIANS, UNIT_TURNS,
    UPDATE_FULL_GRADIENT, UPDATE_SCS,
    Batch, CosmError, Params, State, TTSResult,
    build_partitions, default_params, exported_symbols, lds_probe, library_path, load_library,
    qubo_to_ising, version,
)
