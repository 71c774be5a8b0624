"""MI355X (gfx950) Frequency-Splitting MLMC trace estimation: Python binding.

The compute path is the HIP library libfsmlmc.so (see include/fsmlmc.h); this
package only marshals arguments to it.  Importing `paper_2212_04430_amd.lib`
fails loudly if the library is not built.
"""

import importlib


def lib():
    """The ctypes binding module (raises ImportError if the library is missing)."""
    return importlib.import_module("paper_2212_04430_amd._lib")
