"""CPU oracle for the batched skip-list index -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import anything from this package.  The GPU library never
links, loads or calls it, and the two share no source, header, table or
helper.

Contents
--------
skiplist.c     plain single-threaded Pugh skip list applying queries in arrival
               order (the serial execution the paper's batched processing must
               reproduce, Section 3.2 and Section 4.2), plus the interception of
               Definition 4 and a structural self-check.
skiplist.py    ctypes wrapper (``SkipList``) around the compiled C library.
mapref.py      the same semantics written as a plain map replay (Python dict /
               sorted numpy arrays) for sizes where the C list would be slow.
redistribute.py  Algorithm 3 (hand-over of queries between neighbouring
               workers) written out in Python, with the latch-free invariant of
               Section 3.2.4 as a checker.
build.py       compiles skiplist.c with gcc into ``liborc.so``.
"""
