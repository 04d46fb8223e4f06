"""MI355X-native generalised geodesic distance transform (GGDT).

The compute path is the HIP library ``libggdt.so`` (built from ``csrc/``); the
functions below marshal torch tensors into its C ABI.  They are resolved lazily
so that importing the input generators (``synth``) does not load the library;
calling any of them without a built library raises at once.
"""
_PUBLIC = ("ggdt2d", "ggdt3d", "ggdt_forward_rec", "ggdt_backward", "ggdt_batched", "BatchedPlan",
           "GGDTFunction", "load_library", "GGDTError")


def __getattr__(name):
    if name in _PUBLIC:
        from . import binding
        return getattr(binding, name)
    raise AttributeError(name)


__all__ = list(_PUBLIC)
