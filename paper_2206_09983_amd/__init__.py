"""MI355X (gfx950) streaming subgraph matcher.

The matching runs in the HIP library ``libmnemonic.so`` (sources in ``csrc/``,
C ABI in ``include/mnemonic.h``); ``binding`` is its ctypes binding and
``synth`` draws seeded synthetic graphs, streams and queries. Importing the
package does not load the library; ``binding.load()`` does, and fails loudly
when it has not been built.
"""
