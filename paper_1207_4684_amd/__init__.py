"""MI355X-native hot path of Fast Cauchy Transform l1 regression (arXiv 1207.4684).

``paper_1207_4684_amd.fctl1`` binds the HIP library ``libfctl1.so`` (C ABI in
``include/fctl1.h``); ``paper_1207_4684_amd.build`` compiles it for gfx950.
Importing this package does not load the library.
"""
