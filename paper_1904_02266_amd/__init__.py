"""MI355X-native continuous sensor registration (kernel inner-product
registration on SE(3), Ghaffari et al.).

The compute path is the HIP library in ``lib/libcvo.so`` behind the C ABI of
``include/cvo.h``; ``Context`` is a thin ctypes binding.  ``synth`` draws
seeded synthetic inputs.
"""
from ._binding import (DOF_R3, DOF_SE2, DOF_SE3, DOF_SO3, CVO_EBUSY, CVO_EDEVICE, CVO_EINVAL, CVO_ENOMEM, CVO_ENOOVERLAP,  # noqa: F401
                       CVO_ENOTFOUND, CVO_OK, CVO_PENDING, Context, CvoError, Params, load,
                       params_planes, params_rgbd, params_table1, quartic_step)
