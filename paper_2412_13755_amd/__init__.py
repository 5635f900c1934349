"""MI355X-native TPC track reconstruction: neighbour finding, cellular-automaton
seeding and Kalman helix fit behind the C-ABI library libtpcreco.so (gfx950).

The Python layer only moves data: every step runs in the library's HIP
kernels, and importing the bindings fails loudly if the library is missing.
"""
__all__ = ["Reco", "RecoConfig", "DeviceFrames", "Seeds", "Tracks", "KalmanChi2", "ReconstructGraph"]


def __getattr__(name):
    if name in __all__:
        from . import reco
        return getattr(reco, name)
    raise AttributeError(name)
