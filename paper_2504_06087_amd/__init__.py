"""MI355X-native FiRE hot path: libfire (HIP, gfx950) and its Python binding.

Import ``paper_2504_06087_amd.fire`` for the binding; it loads libfire.so and
fails loudly when the library has not been built.
"""
