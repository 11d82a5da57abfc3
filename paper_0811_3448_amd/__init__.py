"""MI355X (gfx950) stable binar sort: Python binding of libbinar.so.

Gilreath's binar sort orders keys by their bit strings, most significant bit
first, partitioning on each bit (sections "Algorithm Synopsis" and
"Operation of Algorithm").  This package calls the HIP library that does it
on the GPU with stable partitions, k bits per breadth-first pass, a
decoupled look-back scan and an LDS finish; see ``include/binar.h`` for the
C ABI.  The binding only marshals arguments: torch tensors supply device
memory and streams, every step of the sort runs in the library's kernels.
"""
from .binar import (  # noqa: F401
    BINAR_EDEVICE,
    BINAR_EINVAL,
    BINAR_ENOMEM,
    BINAR_ERANGE,
    BINAR_OK,
    KEY_FLOAT,
    KEY_SIGNED,
    KEY_UNSIGNED,
    BinarError,
    Params,
    Plan,
    Workspace,
    default_params,
    key_bytes_of,
    lib,
    profile_enable,
    profile_read,
    resolve_params,
    set_default_params,
    sort,
    sort_inplace,
    inplace_workspace_bytes,
    sort_segmented,
    sort_strings,
    stats,
    strerror,
    strings_workspace_bytes,
    workspace_bytes,
)
