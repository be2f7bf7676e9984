"""CPU oracle of the ENO-AO method -- test infrastructure only (see oracle/enoao_ref.h)."""
