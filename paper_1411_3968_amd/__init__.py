"""MI355X-native hot path of the online muon trigger (arXiv:1411.3968).

The compute runs in ``libtrig.so`` (hand-written HIP for gfx950, C ABI in
``include/trig.h``); :mod:`.trig` is its thin ctypes binding.  Importing
:mod:`.trig` fails loudly when the library is not built.
"""
__all__ = ["trig", "build"]
