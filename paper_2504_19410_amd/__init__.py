"""MI355X-native far-field smooth approximation (FSA) convolution solver.

Hot path of Liu & Zhang, "Fast convolution solver based on far-field smooth
approximation" (arXiv 2504.19410): a once-per-plan FP64 kernel tensor and a
fused zero-padded FFT convolution per evaluation, as hand-written HIP kernels
for gfx950 behind the C ABI of ``include/fsa.h``.

The binding (``paper_2504_19410_amd.fsa``) loads ``libfsa.so`` on import and
raises if it has not been built; ``synth`` holds the seeded input generators.
"""

__all__ = ["fsa", "synth", "build"]
