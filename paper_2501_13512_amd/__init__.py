"""MI355X-native block-preconditioned VIE-FFT solver (arXiv 2501.13512).

The product is ``libvie.so`` (HIP, gfx950) with the C ABI of
``include/vie.h``; ``paper_2501_13512_amd.vie`` is its Python binding.
Build with ``python -m paper_2501_13512_amd.build``.
"""
