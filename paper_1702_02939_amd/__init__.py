"""MI355X-native self-propelled Voronoi (SPV) vertex-model step.

The hot path (periodic Delaunay validity test and device-side repair, Voronoi
geometry, chain-rule forces, active Brownian update) is hand-written HIP for
gfx950 behind the C-ABI declared in ``include/spv.h`` (``libspv.so``).
``paper_1702_02939_amd.spv`` is the thin ctypes binding; ``inputs`` holds the
seeded synthetic workload generators.  Importing this package loads nothing.
"""
