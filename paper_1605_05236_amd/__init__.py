"""MI355X-native batched cuckoo hash tables with the kick-out eviction schemes
of Kuszmaul, "Fast Concurrent Cuckoo Kick-out Eviction Schemes for
High-Density Tables" (arXiv 1605.05236).

The compute path is the HIP library ``libck.so`` (C ABI, declared in
``include/ck.h``); :mod:`.table` is its thin ctypes binding.  Importing this
package loads nothing; the library is opened on first use.
"""
