"""MI355X-native hot path of the p2r / p2z track-fit mini-apps.

Python binding of libp2r.so (include/p2r.h): argument marshalling only.
Every step of the fit runs in the library's HIP kernels; PyTorch provides
device memory and streams.  The library must have been built
(``python paper_2401_14221_amd/build.py``); importing the binding without it,
or calling it without a GPU, raises instead of falling back to anything.
"""
from ._lib import (  # noqa: F401
    P2R_OK, P2R_EINVAL, P2R_ELAYOUT, P2R_EHIP, P2R_ENOTUNED, P2R_ENOSPACE, P2R_MAX_HITS, P2R_NOALLOC_MAX_TRACKS,
    ST_NO_CROSSING, ST_NEWTON_FAIL, ST_FP64_FALLBACK, ST_S_NOT_PD, ST_BAD_INPUT,
    ST_ML_REJECTED, ST_HIT_MISSING, ST_CHI2_CUT, ST_DONE, P2RError, Opts, Context, Mlp,
    library, library_path, exported_symbols, variant_names, device_allocations,
)
from .layout import (  # noqa: F401
    pack_tracks, unpack_tracks, pack_hits_p2r, pack_hits_p2z, n_blocks,
)
