"""MI355X-native validating UTF-8 <-> UTF-16LE transcoding (gfx950 HIP kernels
behind a C-ABI; see include/hiputf.h). The binding is loaded on first use."""
from __future__ import annotations

import importlib

_API = ("validate_utf8", "utf16_length_from_utf8", "convert_utf8_to_utf16le",
        "validate_utf16le", "utf8_length_from_utf16le", "convert_utf16le_to_utf8")


def __getattr__(name):
    if name in _API or name in ("binding",):
        mod = importlib.import_module(".binding", __name__)
        return mod if name == "binding" else getattr(mod, name)
    raise AttributeError(name)
