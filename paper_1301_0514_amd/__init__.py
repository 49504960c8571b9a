"""MI355X (gfx950) phase-screen + Fresnel propagation library for the method
of Habibi, Moniez, Ansari & Rahvar, "Simulation of optical interstellar
scintillation" (A&A 2013).  The kernels live in lib/libscint.so (build with
`python -m paper_1301_0514_amd.build`); paper_1301_0514_amd.scint binds them."""

__all__ = ["scint", "presets"]
