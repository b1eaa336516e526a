"""MI355X-native BP + localized statistics decoding (LSD).

The decoder itself lives in the HIP library ``libqlsd.so`` (sources under
``csrc/``); ``binding`` is a thin ctypes layer over its C ABI.  Importing this
package does not load the library; ``binding.lib()`` does, and fails loudly when
it has not been built.
"""
