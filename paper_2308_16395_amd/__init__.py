"""Streaming Tucker (streaming ST-HOSVD) on AMD MI355X (gfx950).

The compute path is the C ABI library libstucker.so (include/stucker.h);
``binding`` marshals arguments to it. Importing the package loads the library
and raises if it has not been built.
"""

from .binding import (  # noqa: F401
    EXPORTED,
    LIB_PATH,
    StError,
    StreamingTucker,
    lib,
)
