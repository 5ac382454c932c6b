"""Seeded, slice-replayable synthetic streams.

This module only produces input data. It holds none of the streaming Tucker
arithmetic, so both the FP64 CPU oracle (through the tests) and the GPU path
(through the tests and the benchmark) can draw the same inputs from it.

Every generator draws its parameters once from ``numpy.random.default_rng(seed)``
and then produces slice ``t`` as a pure function of (parameters, t). A slice of a
stream with slice dims (n_1, ..., n_{d-1}) is returned as a float64 array of that
shape in Fortran (column-major) order: the first index is fastest, which is the
memory order of a mode-1 fibre (paper section 2.1, matricization).
"""

from .generators import (  # noqa: F401
    LowRankStream,
    BlobStream,
    FourierStream,
    SineWaveTensor,
    SineWaveStream,
    SINE_WAVE,
    make_stream,
    CONFIGS,
)
