"""MI355X-native four-way coupled lattice Boltzmann / discrete element method
(Rettinger & Ruede, arXiv:2003.01490): HIP kernels for gfx950 behind the C-ABI
of ``include/lbmdem.h``, with a thin ctypes binding in :mod:`.lbmdem`."""
from . import lbmdem  # noqa: F401
from .lbmdem import Config, Domain, LbmdemError, default_config, footprint_bytes  # noqa: F401
