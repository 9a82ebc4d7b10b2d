"""scaletrack for MI355X: the per-particle Lagrangian time step of SCALE-TRACK
(arXiv 2603.26691) as hand-written HIP kernels behind a C ABI (include/st.h).

The HIP library is loaded on first use; importing this package does not
touch the GPU.
"""


def __getattr__(name):
    if name == "Tracker":
        from .tracker import Tracker
        return Tracker
    if name == "DepositFn":
        from .autograd import DepositFn
        return DepositFn
    raise AttributeError(name)
