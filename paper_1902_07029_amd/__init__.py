"""MI355X-native level-set multigrid for the sulfation model (arXiv 1902.07029).

The compute path is the HIP library ``liblsmg.so`` (sources in ``csrc/``, C ABI in
``include/lsmg.h``); ``lsmg`` is its Python binding.  Importing this package does
not load the library; ``paper_1902_07029_amd.lsmg.load()`` does, and fails if the
library has not been built.
"""
