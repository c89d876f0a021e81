"""MI355X-native all-pairs Stokesian-dynamics mobility product (HIP, gfx950).

The compute path lives in the HIP shared library built from ``csrc/``; the
Python functions here only marshal arguments to its C ABI.  Importing the
package does not load the library; the first call does, and fails loudly if
the library is missing.
"""
