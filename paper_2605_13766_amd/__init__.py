"""MI355X-native discrete Cosserat-rod step (HIP for gfx950 behind a C ABI).

Submodules are imported lazily: ``workloads`` (seeded synthetic inputs) needs
only numpy; ``rod`` (the binding of ``librod.so``) needs the built library.
"""
