"""MI355X-native error-bounded lossy compressor for N-body particle fields.

The compute path is the HIP library ``csrc/libsznb.so`` (C ABI declared in
``include/sznb.h``); ``sznb`` is its thin ctypes binding.  Importing the
package does not load the library: the first call does, and fails loudly if
it has not been built.
"""
