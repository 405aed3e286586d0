"""MI355X-native fast proper orthogonal descriptors (POD).

The compute path is the HIP library ``libpod.so`` (C ABI declared in
``include/pod.h``); ``paper_2212_14446_amd.pod`` is its thin Python binding.
Importing this package loads nothing; the library is loaded on first use.
"""
