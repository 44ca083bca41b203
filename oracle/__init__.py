"""FP64 CPU oracle for the Fourier-domain acceleration search (FDAS).

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package. The product path (the
HIP library and its Python binding) never imports, links or calls it, and the
oracle shares no code, table or constant generator with that path.

Every function states the plain definition it computes. The paper
(Section 2, pipeline steps 3-5: realfft, accelsearch, candidate sifting; the
zmax knob of Section 3.2 and Table 4) names these steps but does not define
their mathematics; the definitions below are the readings adopted for it and
are listed, one by one, with the design notes of the repository.
"""
from .fdas_oracle import *  # noqa: F401,F403
from .fdas_oracle import __all__  # noqa: F401
from .refine_oracle import *  # noqa: F401,F403
from .refine_oracle import __all__ as _refine_all  # noqa: F401

__all__ = list(__all__) + list(_refine_all)
from .dedisp_oracle import *  # noqa: F401,F403
from .dedisp_oracle import __all__ as _dedisp_all  # noqa: F401

__all__ = list(__all__) + list(_dedisp_all)
from .sift_oracle import *  # noqa: F401,F403
from .sift_oracle import __all__ as _sift_all  # noqa: F401

__all__ = list(__all__) + list(_sift_all)
