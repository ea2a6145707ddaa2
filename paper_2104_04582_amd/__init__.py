"""MI355X-native interpolated harmonic-mode summation (FastEMRIWaveforms-style).

The compute path lives in the HIP library built from ``csrc/`` (``libfew.so``);
``native`` is its thin ctypes binding.  ``synth`` draws seeded inputs.
"""
