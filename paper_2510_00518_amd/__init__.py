"""MI355X-native three- and four-phonon scattering rates.

The compute path lives in the C-ABI library built from ``csrc/`` (``libfp.so``);
``fp`` is its Python binding.  ``synth`` builds seeded synthetic inputs.
"""
