"""Yin-Yang multipole gravity on MI355X (gfx950).

`paper_1806_04593_amd.yyg` is the thin ctypes binding of the C-ABI library
built from `csrc/`; `paper_1806_04593_amd.workloads` makes the seeded
synthetic density fields.  Importing the package loads neither.
"""
