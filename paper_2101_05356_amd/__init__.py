"""MI355X-native differentiable face render (Dib et al., "Practical Face
Reconstruction via Differentiable Ray Tracing", Eurographics 2021).

The compute lives in libfr.so (HIP, gfx950) behind the C ABI of include/fr.h;
`render` wraps it for PyTorch tensors, `scenes` generates seeded synthetic
inputs.  Submodules are imported lazily so that the scene generators load
without a GPU.
"""
import importlib

__all__ = ["render", "scenes", "build"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f".{name}", __name__)
    raise AttributeError(name)
