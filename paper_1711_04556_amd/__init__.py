"""MI355X (gfx950) tabu search for the RCPSP after Bukata, Sucha & Hanzalek.

The compute path is the HIP library librcpsp.so behind include/rcpsp.h;
`paper_1711_04556_amd.rcpsp` is its Python binding and
`paper_1711_04556_amd.synth` generates seeded synthetic instances.
"""
