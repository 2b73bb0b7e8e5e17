"""MI355X (gfx950) checkerboard Metropolis sweep for lattice spin models.

Hot path of "Simulating lattice spin models on GPUs" (Levy, Cohen & Rabani,
arXiv:1209.0296): sub-lattice-parallel Metropolis sweeps of the spin-1/2 and
spin-1 Ising model in 2D/3D and of the North-East facilitated model (also by
the paper's random sub-lattice algorithm, and with the Ising coupling), in
hand-written HIP kernels behind the C ABI of ``include/spinlat.h``.
"""
from .spinlat import (  # noqa: F401
    ABI_VERSION, EXPORTS, INIT_BUFFER, INIT_COLD, INIT_RANDOM, ISING, MODE_AUTO, MODE_FUSED,
    MODE_HALF, MODE_HALF_ROWS, MODE_HALF_WINDOW, MODE_FUSED_WINDOW, MODE_RESIDENT, MODE_SIMPLE, NORTH_EAST,
    NE_COUPLED, NE_SUBLATTICE, NE_SUBLATTICE_BALANCED, RECORD_DTYPE, Lattice, Params, SpinlatError, lib,
    query_bytes, records_to_array, threshold_table, Batch, batch_config, batch_job_bytes,
    batch_base_bytes, record_statistics, autocorrelation, BATCH_NO_GRAPH, BATCH_NO_FUSED,
    BATCH_NO_RESIDENT,
)
