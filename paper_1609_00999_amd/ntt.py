"""Python binding of the transform entry points of libmont (argument marshalling only)."""
from __future__ import annotations


def register(L) -> None:
    """Declare ctypes argument types for the transform entry points."""
    return None
