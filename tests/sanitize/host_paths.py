"""Host-side paths of the HIP library that need no device, under
AddressSanitizer + UndefinedBehaviorSanitizer (started by
tests/test_sanitizers.py): parameter validation and workspace sizes over
random parameter sets, the saved-state checker over random and corrupted
blobs, and the name and error queries."""
import os
import struct
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
from paper_2504_12858_amd import binding as B  # noqa: E402

lib = B.load_library(sys.argv[1])
import ctypes as C  # noqa: E402

rng = np.random.default_rng(7)
ok = 0
base = dict(lo=(0.0, 0.0, 0.0), hi=(1e-3, 1e-3, 2e-3), lambda0=5e-6, h=10e-6, rc=5e-6,
            a=(1e-5, 1e-6), b=(2.0, 3.0), theta=0.0, cap_particles=1 << 16, cap_stopped=1 << 16,
            cap_grains=1 << 12, cap_sites=64, cap_claim_bricks=1 << 12, field_n=(0, 0, 0),
            resort_every=0, periodic=0)
choices = dict(lo=[(-1e-3, 0.0, 0.0), (np.nan, 0.0, 0.0)], hi=[(1e-3, 0.0, 1e-3), (1.0, 1.0, 1.0)],
               lambda0=[1e-6, 0.0, -1.0, np.nan, 1e-9], h=[5e-6, 2e-6, 0.0, np.inf],
               rc=[2.5e-6, 20e-6, 0.0], a=[(-1e-5, 0.0), (np.inf, 0.0)], b=[(2.7, 1.5), (np.nan, 2.0)],
               theta=[np.nan, 1.0], cap_particles=[0, 5, 6, 1 << 40],
               cap_stopped=[0, 1, 1 << 33], cap_grains=[0, 1, (1 << 28) - 2, 1 << 28],
               cap_sites=[-1, 0], cap_claim_bricks=[0, 1, 1 << 31, 1 << 32],
               field_n=[(1, 2, 2), (2, 2, 2), (256, 256, 256), (-1, 0, 0)],
               resort_every=[-1, 1, 1 << 30], periodic=[3, 7, 8, -1])
for k in range(3000):
    args = dict(base)
    for key in rng.choice(list(choices), size=int(rng.integers(0, 3)), replace=False):
        opts = choices[key]
        args[key] = opts[int(rng.integers(0, len(opts)))]
    p = B.make_params(**args)
    n = C.c_size_t()
    rc1 = lib.ge_validate_params(C.byref(p))
    rc2 = lib.ge_workspace_size(C.byref(p), C.byref(n))
    assert rc1 == rc2
    ok += rc1 == 0
assert 0 < ok < 3000, ok
lib.ge_validate_params(None)
for k in range(-2, 20):
    lib.ge_phase_name(k)
    lib.ge_tunable_name(k)
assert lib.ge_last_error(None) is not None
# Saved-state checker: random bytes, truncations, corrupted headers.
hdr = struct.Struct("<IIQQd3d3ddqqqqq")
for k in range(400):
    n = int(rng.integers(0, 600))
    blob = rng.integers(0, 256, n, dtype=np.uint8)
    if n >= hdr.size and k % 2:
        counts = rng.integers(-2, 4, 4)
        payload = n - hdr.size
        blob[:hdr.size] = np.frombuffer(hdr.pack(0x54534547, 1, n, 0, 5e-6, 0, 0, 0, 1, 1, 1, 0.0,
                                                 0, *[int(c) for c in counts]), np.uint8)
    h = B.ge_state_header()
    lib.ge_state_check(blob.ctypes.data_as(C.c_void_p), blob.nbytes, C.byref(h))
lib.ge_state_check(None, 0, None)
print("host paths clean", flush=True)
