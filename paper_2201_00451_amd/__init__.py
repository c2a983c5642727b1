"""MI355X-native resampling F-statistic (arXiv:2201.00451 method).

The compute path is a HIP library for gfx950 behind a C ABI
(``include/fstat.h``); ``binding`` marshals torch device tensors into it.
``synth`` builds seeded synthetic inputs.
"""
