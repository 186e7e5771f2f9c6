"""MI355X-native evaluation of Boolean terms on free Boolean generators.

The compute path is the HIP library libfbg.so (include/fbg.h); this package
is its ctypes binding.  Importing it fails loudly when the library has not
been built.
"""

from .fbg import (  # noqa: F401
    Batch,
    FbgError,
    Program,
    as_u64,
    compile,
    compile_assume,
    compile_subst,
    count,
    count_batch,
    dnf_words,
    enumerate_dnf,
    enumerate_models,
    eval_dnf,
    program_tiles,
    Server,
    version,
)
