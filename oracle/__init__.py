"""CPU oracle for longest-prefix match -- test infrastructure, not product code.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import or run anything in this package.  It shares no code,
header, table or helper with the GPU library (``paper_2604_14650_amd``) and
never imports it.

What it computes is the plain definition of the problem the paper solves
(Background, "IPv6 Prefix Length and Distribution"; Design, "From 2D Prefixes
to 1D Intervals"): for a destination x, the next hop of the rule (P, L) whose
top L bits equal x's top L bits with L maximal (L = 0 always matches); if no
rule matches, the reserved value NO_ROUTE = 0xFFFF (the paper's "-1" / default
route when no ::/0 exists).

* ``brute``  -- scans every rule per address (Python ints; numpy variant).
* ``trie``   -- a textbook one-bit-per-level binary trie in plain C
                (``trie.c``), multithreaded over addresses.
* ``mlp``    -- float64 forward/backward/Adam of the learned position model.
"""
NO_ROUTE = 0xFFFF
