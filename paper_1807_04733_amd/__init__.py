"""MI355X-native hot-electron particle-in-cell step (Nenno, Rethfeld, Schneider,
arXiv:1807.04733): hand-written HIP kernels for gfx950 behind a C ABI (libpic.so),
with a thin ctypes binding.  Importing the package does not load the library; the
first PicSim does, and fails loudly if it has not been built."""
from ._abi import COUNTER_NAMES, NCOUNTERS, PicError  # noqa: F401


def __getattr__(name):
    if name in ("PicSim", "make_config", "workspace_bytes"):
        from . import sim
        return getattr(sim, name)
    raise AttributeError(name)
