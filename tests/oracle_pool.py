"""Oracle runs in worker processes (spawned, so they never touch the GPU)."""


def oracle_export(c):
    """Run circuit ``c`` through the map oracle; (keys[n, 4], amps[n])."""
    from oracle.oracle import run_circuit
    st, _, _ = run_circuit(c)
    k, _, a = st.export()
    return k, a
