"""The graph the decoder library holds, as the graph object the oracle
takes: every GPU-against-oracle comparison decodes the table read back from
the library (ldpc_get_graph), so both sides decode the same graph."""
import numpy as np

from synth import BaseGraph, make_graph


def library_graph(bg: int, Z: int, rows: int | None = None) -> BaseGraph:
    """Register the seeded graph (bg, Z) with the library if it is not, read
    it back through ldpc_get_graph and keep the first ``rows`` block rows."""
    from paper_2009_05534_amd import ldpc
    try:
        m_rows, kb, row, col, shift = ldpc.get_graph(bg, Z)
    except ldpc.LdpcError:
        ldpc.register(make_graph(bg, Z))
        m_rows, kb, row, col, shift = ldpc.get_graph(bg, Z)
    counts = np.bincount(row.astype(np.int64), minlength=m_rows)
    row_ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    g = BaseGraph(bg=bg, Z=Z, M=m_rows, N=kb + m_rows, kb=kb, row_ptr=row_ptr,
                  col=col.astype(np.int16), shift=shift.astype(np.int16))
    return g if rows is None or rows == m_rows else g.sub(rows)
