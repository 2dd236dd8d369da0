"""MI355X (gfx950) hologram-rendering hot path: angular-spectrum / Fresnel
reconstruction, short-time DFT Doppler moments and PCA, as hand-written HIP
kernels behind the C-ABI in include/hv.h.

``paper_2508_03911_amd.hv`` is the Python binding; importing it loads the
in-tree ``libhv.so`` (built by ``paper_2508_03911_amd.build``) and fails if it
is absent.
"""

import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libhv.so")
