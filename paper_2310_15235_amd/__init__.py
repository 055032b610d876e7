"""MI355X (gfx950) implementation of the TREVR2 radiative-transfer hot path
(Wadsley, Baumschlager & Shen 2023): tree build, per-bucket HEALPix walk,
ray reduction and p-p near field as HIP kernels behind the C ABI in
include/trevr2.h.  ``api`` is the Python binding; ``scenes`` the seeded
input generators."""
from . import scenes  # noqa: F401

__all__ = ["scenes", "api"]


def __getattr__(name):
    if name == "api":
        import importlib
        return importlib.import_module(".api", __name__)
    raise AttributeError(name)
