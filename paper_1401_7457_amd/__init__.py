"""cxbwt: multi-string BWT construction for short-read collections on MI355X.

The device path lives in the HIP library ``libcxbwt.so`` (sources under
``csrc/``); ``cxbwt.py`` is its thin Python binding.  Importing this package
does not load the library; the first call into the binding does, and fails
loudly when the library has not been built.
"""

__all__ = ["cxbwt", "datagen"]
