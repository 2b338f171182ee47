"""MI355X-native Neural Bootstrapping Method hot path.

`binding.NBM` wraps the C ABI of libnbm.so (include/nbm.h); `train` holds the
torch autograd wrapper and the training loop built on it.
"""
from .binding import NBM, NbmError, lib  # noqa: F401
