"""MI355X (gfx950) treecode for 3D Stokeslets and stresslets (Wang, Tlupova & Krasny,
arXiv 1811.12498).  The HIP library is loaded lazily by ``paper_1811_12498_amd.native``;
``workloads`` (seeded input generators) imports no GPU code."""

__all__ = ["native", "workloads"]


def __getattr__(name):
    if name == "native":
        from . import _native as native
        return native
    raise AttributeError(name)
