"""MI355X-native MRTLB-VANSE: the D2Q9 collide-and-stream step of the
consistent multiple-relaxation-time lattice Boltzmann method for the
volume-averaged Navier-Stokes equations, as one fused HIP kernel for gfx950
behind a C-ABI library (``libvanse.so``).

``paper_2409_02964_amd.vanse`` is the Python binding (argument marshalling
only); ``paper_2409_02964_amd.workloads`` builds seeded synthetic inputs.
"""
__all__ = ["vanse", "workloads"]
