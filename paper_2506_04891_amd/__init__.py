"""MI355X-native batched state-vector simulator for layered QML circuits.

The simulation runs in ``libtqsim.so`` (HIP kernels for gfx950 behind a C ABI,
``include/tqsim.h``); ``tqsim`` is its ctypes binding with a
``torch.autograd.Function`` wrapper; ``serve`` is the continuous-batching
request loop.
"""
from .tqsim import Circuit, QCircuitFn, TqsError, expval, lib  # noqa: F401
