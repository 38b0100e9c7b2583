"""MI355X-native stereo matching after Chang & Maruyama (arXiv 2212.00488).

``binding`` holds the ctypes front end of the C interface (include/stereo.h);
``synth`` the seeded synthetic stereo pairs; ``build`` the hipcc build.
Importing the package loads nothing; the library is loaded on first use.
"""

from .binding import (EHIP, EINVAL, ENOMEM, F_FULL_RES, F_KEEP_INTERMEDIATES,  # noqa: F401
                      F_STAGE_TIMING, OK, STAGES, Params,
                      Stereo, StereoError, default_params, lib)
