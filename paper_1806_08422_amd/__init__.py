"""MI355X-native noisy mean-field annealing (NMFA).

The hot path of King et al., "Emulating the coherent Ising machine with a mean-field algorithm"
(arXiv:1806.08422, Algorithm 1) as hand-written HIP kernels for gfx950 behind a C ABI
(include/nmfa.h, libnmfa.so). ``paper_1806_08422_amd.nmfa`` is the Python binding; importing it
loads the library and fails if it has not been built.
"""

__all__ = ["nmfa"]


def __getattr__(name):
    if name == "nmfa":
        import importlib

        return importlib.import_module(".nmfa", __name__)
    raise AttributeError(name)
