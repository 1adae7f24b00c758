"""FP64 CPU oracle of the operator-splitting PPML update (arXiv:1607.01105).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU
product path never imports, links or executes anything here, and this
package imports nothing from the product package.
"""
from .oracle import (Oracle, avg_left, avg_right, build, lib_path, load_library, max_threads,  # noqa: F401
                     multipole_value, reconstruct_line, set_threads, sine_transform)
