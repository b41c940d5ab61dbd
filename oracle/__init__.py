"""CPU reference for the local block-sparse multiply -- TEST INFRASTRUCTURE ONLY.

Imported only by ``tests/``, the smoke check and the benchmark's
CPU-baseline leg.  It shares no code with the GPU library and imports
nothing from it.
"""
