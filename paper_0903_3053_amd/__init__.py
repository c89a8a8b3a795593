"""SU(2) Wilson-action heat-bath sweep on MI355X (gfx950): a HIP library with a
C ABI (include/su2.h) and a thin ctypes binding (su2.py).

Method: Demchik & Strelchenko, arXiv:0903.3053, Sec. 2.4.
"""
from . import su2  # noqa: F401
from .su2 import (COLD, HOT, Su2Error, su2_counters, su2_finalize, su2_init, su2_init_ex,  # noqa: F401
                  su2_links, su2_measure_device, su2_pass, su2_philox, su2_plaquette, su2_plaquette_st, su2_polyakov,
                  su2_set_links, su2_set_plan, su2_set_stream, su2_tune, su2_sweep, su2_sweep_index, su2_sweep_measure,
                  su2_sweep_measured,
                  su2_synchronize)
