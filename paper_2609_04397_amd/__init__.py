"""MI355X-native variable-block sparse products (VBCSR hot path).

``Matrix`` / ``spmm`` load the HIP library and torch on first use; importing
the package itself touches neither.
"""

__all__ = ["Matrix", "spmm", "spmm_pages", "Halo", "VbcsrError"]


def __getattr__(name):
    if name in ("Matrix", "spmm", "spmm_pages"):
        from . import matrix
        return getattr(matrix, name)
    if name == "Halo":
        from .halo import Halo
        return Halo
    if name == "VbcsrError":
        from ._lib import VbcsrError
        return VbcsrError
    raise AttributeError(name)
