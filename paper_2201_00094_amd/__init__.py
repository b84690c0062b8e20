"""MI355X-native wavelet-transparency resolve (Wavelet Transparency, Aizenshtein, Smal, McGuire 2021).

The compute lives in ``libwt.so`` (HIP kernels for gfx950 behind the C ABI of ``include/wt.h``); this package
marshals torch tensors into it. Importing it does not load the library; the first call does, and fails loudly
if the library has not been built.
"""
from ._lib import WTError, load as load_library  # noqa: F401
from .wt import (FrameSpec, Fragments, Workspace, backward, bin, bin_count, bin_scatter, build,  # noqa: F401
                 build_binned, dropped_count, evaluate, evaluate_binned, render, render_binned, render_noalloc,
                 render_temporal, render_temporal_binned, resolve, resolve_chromatic, workspace_bytes)
from .autograd import WaveletComposite, composite  # noqa: F401
