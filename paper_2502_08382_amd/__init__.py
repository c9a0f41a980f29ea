"""fetiF: explicit FETI local dual operators on AMD Instinct MI355X.

The computation lives in the in-tree shared library ``libfetiF.so`` (C++
host analysis + HIP kernels for gfx950) behind the C-ABI of
``include/fetiF.h``; this package only marshals arguments.
"""
from .fetif import (FetiContext, FetiError, HostFactor, load_library, LIB_PATH,  # noqa: F401
                    F64, F32, BF16)
from .problem import subdomain_dict, values_in_pattern  # noqa: F401
