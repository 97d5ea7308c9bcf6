"""MI355X (gfx950) factored extrinsic likelihood and its Monte-Carlo evidence.

    from paper_2609_37393_amd import ile      # HIP library binding (torch + ctypes)
    from paper_2609_37393_amd import synth    # seeded synthetic inputs

The binding is imported lazily so that the light-weight modules (synth, build)
do not pull in torch.
"""

__all__ = ["ile", "synth", "build"]


def __getattr__(name):
    if name in __all__:
        import importlib

        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
