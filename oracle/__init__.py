"""FP64 CPU oracle for the streaming ST-HOSVD update (test infrastructure).

This package is the plain, slow reference that the GPU library is checked
against. It is test infrastructure: only the test suite, the smoke check in
``__graft_entry__`` and the ``cpu_baseline`` leg of ``bench.py`` may import it.
The product path never imports, calls or links anything here, and nothing
here imports the product package.
"""

from .tucker import (  # noqa: F401
    unfold,
    fold,
    ttm,
    multi_ttm,
    reconstruct,
    tsvd_gram,
    sthosvd,
    isvd,
    block_isvd,
    non_streaming_update,
    StreamingTucker,
    vec,
)
from .grad import (  # noqa: F401
    tucker_reconstruct,
    tucker_reconstruct_loss_grad,
    tucker_project,
    tucker_project_vjp,
)
