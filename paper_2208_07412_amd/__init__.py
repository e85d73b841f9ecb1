"""MI355X-native TPC track reconstruction (clusterization, cellular-automaton
neighbour finding, tracklet seeding, Kalman following and refit).

The reconstruction runs in the HIP kernels of ``libtpcreco.so`` behind the C
ABI of ``include/tpc.h``; ``paper_2208_07412_amd.tpc`` is its Python binding.
"""
from . import build  # noqa: F401
