"""MI355X (gfx950) range-discord search: MERLIN over a length range with
parallel DRAG-style selection and refinement sweeps, behind a C ABI.

The public entry points live in :mod:`paper_2304_01660_amd.api`; importing
them loads ``libpalmad.so`` (built in-tree) and needs torch.
"""

__all__ = ["api", "synth"]
