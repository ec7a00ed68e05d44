"""MI355X-native hot path of proxy-sampling BDPT (Su et al., Proxy Tracing, arXiv 2503.23412).

The rendering path lives in libpt.so (HIP, gfx950) behind the C ABI of include/pt.h; pt.py is
the ctypes binding.
"""
from . import pt  # noqa: F401
