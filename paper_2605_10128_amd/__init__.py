"""MI355X (gfx950) batched DC N-1 topology screen for MapElites transmission
topology optimisation.  The compute path is the HIP library libtto.so behind
the C ABI in include/tto.h; ``paper_2605_10128_amd.tto`` is its ctypes
binding.  Submodules are imported lazily so that building does not need the
library to exist yet."""

__all__ = ["tto", "screen", "build"]
