"""MI355X-native fast force-coupling method (fast FCM) mobility.

The computation lives in the HIP library ``libfcm.so`` (C ABI in
include/fcm.h); this package is its thin Python binding.
"""

from ._lib import (FCM_EDEVICE, FCM_EINVAL, FCM_ENOMEM, FCM_ENONFINITE, FCM_ERANGE, FCM_ESCRATCH,
                   FCM_FP32_BULK, FCM_FP64, FCM_OK, EXPORTS, STAGES, FCMError, LibraryMissing, Options,
                   Plan, fcm_options_default, fcm_plan_footprint, library, mobility_static, status_string,
                   LIB_PATH)

__all__ = ["Plan", "FCMError", "LibraryMissing", "Options", "library", "status_string",
           "fcm_options_default", "fcm_plan_footprint", "FCM_FP64", "FCM_FP32_BULK", "FCM_OK",
           "FCM_EINVAL", "FCM_ENOMEM", "FCM_EDEVICE", "FCM_ERANGE", "FCM_ENONFINITE", "FCM_ESCRATCH", "mobility_static", "EXPORTS",
           "LIB_PATH", "STAGES"]
