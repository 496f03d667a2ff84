"""MI355X-native black-box randomized compression of HBS matrices.

The hot path (the level-by-level compression sweep of Algorithm 2, the apply
of Algorithm 1 and the log-kernel stand-in black box) is hand-written HIP for
gfx950 in ``csrc/``, exported through the C ABI of ``include/hbs.h`` as
``libhbs.so``; ``hbs`` is its Python binding.
"""
