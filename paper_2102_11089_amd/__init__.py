"""MI355X-native dynamic-schedule LDPC belief-propagation decoder (CIRBP / RBP / ME-CIRBP,
flooding and layered baselines).  The decoding entry points live in ``ldpc`` and load the HIP
library on first use."""
