"""MI355X-native Falcon lossless float codec (arXiv 2511.04140).

The codec itself lives in the HIP library libfalcon.so (C ABI declared in
include/falcon.h).  This package only marshals arguments: torch tensors
provide device memory and the current HIP stream.  Attributes are loaded
lazily so that `paper_2511_04140_amd.workloads` imports without torch.
"""
__all__ = ["Codec", "FalconError", "compress", "decompress", "compress_bound", "lib_path"]


def __getattr__(name):
    if name in __all__:
        from . import codec
        return getattr(codec, name)
    raise AttributeError(name)
