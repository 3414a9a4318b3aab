"""MI355X (gfx950) library for the signal-formation hot path of pixelated LArTPC
simulation (arXiv 2602.12052): effective charge of diffused line depositions,
block-sparse binning, interlaced FFT convolution with the field response and
overlap-add into per-pixel waveforms.

The arithmetic lives in the HIP library ``libtred.so`` (C ABI in include/tred.h);
``tred`` is its thin ctypes binding over torch device tensors.
"""

__all__ = ["tred", "build"]
